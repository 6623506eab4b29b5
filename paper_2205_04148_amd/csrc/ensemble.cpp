// Batched ensemble of independent grids: the acoustic-substep launch sequence
// of every member is recorded once, and each recorded kernel then runs for
// all members in a single launch (member-indexed blocks, arguments from a
// device table).  The kernel boundaries are the stage barriers.  Optionally
// the whole call is captured in a HIP graph and replayed, and the block shape
// of every plane kernel is chosen by timing candidate shapes (an autotuner
// whose choices are cached per kernel and reused wherever the same kernel
// appears again: other stages, other ensembles).
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fv3_internal.hpp"

using fv3::MemberBlk;
using fv3::Site;

namespace {

const dim3 kShapes[] = {dim3(64, 4, 1), dim3(128, 2, 1), dim3(256, 1, 1), dim3(32, 8, 1), dim3(16, 16, 1)};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

// autotuner cache: ensemble kernel -> chosen shape index
std::mutex g_tune_mu;
std::map<const void *, int> g_tune_cache;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct fv3_ensemble {
    int members = 0, n_split = 1, device = 0;
    double dt = 0.0;
    fv3::Recorder rec;
    std::vector<int> shape;         // per site (tunable sites only use it)
    std::vector<dim3> grid;         // per site, for its current shape
    std::vector<size_t> arg_off, tab_off;
    char *dbuf = nullptr;
    bool use_graph = false;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// member table of site s for its current shape; returns the launch grid
dim3 site_table(const fv3_ensemble *e, size_t s, std::vector<MemberBlk> &tab)
{
    const Site &S = e->rec.sites[s];
    dim3 b = S.tunable ? kShapes[e->shape[s]] : S.blk;
    tab.resize(e->members);
    long total = 0;
    for (int m = 0; m < e->members; m++) {
        int x = S.tunable ? (S.ex[m] + (int)b.x - 1) / (int)b.x : S.ex[m];
        int y = S.tunable ? (S.ey[m] + (int)b.y - 1) / (int)b.y : S.ey[m];
        tab[m] = MemberBlk{(int)total, x, y, S.ez[m]};
        total += (long)x * y * S.ez[m];
    }
    // one-dimensional grid: every member's blocks back to back
    return dim3((unsigned)std::max(total, 1L), 1, 1);
}

fv3_status upload_table(fv3_ensemble *e, size_t s)
{
    std::vector<MemberBlk> tab;
    e->grid[s] = site_table(e, s, tab);
    if (hipMemcpy(e->dbuf + e->tab_off[s], tab.data(), tab.size() * sizeof(MemberBlk), hipMemcpyHostToDevice) !=
        hipSuccess)
        return FV3_EDEVICE;
    return FV3_OK;
}

hipError_t launch_site(const fv3_ensemble *e, size_t s, hipStream_t st)
{
    const Site &S = e->rec.sites[s];
    void *dargs = e->dbuf + e->arg_off[s];
    void *dtab = e->dbuf + e->tab_off[s];
    int m = e->members;
    void *kp[] = {&dargs, &dtab, &m};
    dim3 b = S.tunable ? kShapes[e->shape[s]] : S.blk;
    return hipLaunchKernel(S.kmulti, e->grid[s], b, kp, 0, st);
}

hipError_t launch_range(const fv3_ensemble *e, size_t a, size_t b, hipStream_t st)
{
    for (size_t s = a; s < b; s++) {
        hipError_t r = launch_site(e, s, st);
        if (r != hipSuccess) return r;
    }
    return hipSuccess;
}

hipError_t launch_call(const fv3_ensemble *e, hipStream_t st)
{
    const auto &mk = e->rec.marks;
    hipError_t r = launch_range(e, 0, mk[0], st);
    for (int it = 0; it < e->n_split && r == hipSuccess; it++) r = launch_range(e, mk[0], mk[1], st);
    if (r == hipSuccess) r = launch_range(e, mk[1], e->rec.sites.size(), st);
    return r;
}

void drop_graph(fv3_ensemble *e)
{
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    e->exec = nullptr;
    e->graph = nullptr;
}

fv3_status build_graph(fv3_ensemble *e)
{
    drop_graph(e);
    if (hipStreamBeginCapture(e->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fv3::set_error(FV3_EDEVICE, "stream capture failed to start");
    hipError_t r = launch_call(e, e->cap);
    hipError_t r2 = hipStreamEndCapture(e->cap, &e->graph);
    if (r != hipSuccess || r2 != hipSuccess || !e->graph) {
        drop_graph(e);
        return fv3::set_error(FV3_EDEVICE, "capture of the substep sequence failed");
    }
    if (hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0) != hipSuccess) {
        drop_graph(e);
        return fv3::set_error(FV3_EDEVICE, "graph instantiation failed");
    }
    return FV3_OK;
}

bool state_ok(const fv3_state *s, const fv3_grid *g)
{
    if (!s || !g) return false;
    const void *req[] = {s->u, s->v, s->w, s->delp, s->pt, s->delz, s->uc, s->vc, s->mfx, s->mfy,
                         s->cx, s->cy, s->dp0, s->pfull, s->phi, s->workspace};
    for (const void *p : req)
        if (!p) return false;
    return s->workspace_bytes >= g->ws_bytes;
}

}  // namespace

extern "C" {

fv3_status fv3_ensemble_create(fv3_state *const *states, const fv3_grid *const *grids, int members, double dt,
                               int n_split, int flags, fv3_ensemble **out)
{
    if (!states || !grids || !out) return fv3::set_error(FV3_EINVAL, "NULL argument");
    *out = nullptr;
    if (members < 1 || members > 4096) return fv3::set_error(FV3_EINVAL, "members must be in [1, 4096]");
    if (!std::isfinite(dt) || !(dt > 0.0)) return fv3::set_error(FV3_EINVAL, "dt must be finite and positive");
    if (n_split < 1) return fv3::set_error(FV3_EINVAL, "n_split must be >= 1");
    for (int m = 0; m < members; m++) {
        if (!state_ok(states[m], grids[m]))
            return fv3::set_error(FV3_EINVAL, "member " + std::to_string(m) + ": NULL field or small workspace");
        if (grids[m]->bulk_bytes != grids[0]->bulk_bytes)
            return fv3::set_error(FV3_EDTYPE, "all members must share one precision");
        if (!fv3::device_current(grids[m]))
            return fv3::set_error(FV3_EDEVICE, "current HIP device differs from a member's device");
    }
    fv3_ensemble *e = new fv3_ensemble();
    e->members = members;
    e->dt = dt;
    e->n_split = n_split;
    e->use_graph = (flags & FV3_ENSEMBLE_GRAPH) != 0;
    (void)hipGetDevice(&e->device);
    for (int m = 0; m < members; m++) {
        e->rec.member = m;
        fv3_status r = fv3::record_substeps(states[m], grids[m], dt / n_split, &e->rec);
        if (r == FV3_EUNSUPPORTED) {
            delete e;
            return fv3::set_error(r, "member " + std::to_string(m) +
                                         ": its options choose a launch sequence other than member 0's (PPM "
                                         "orders, damping switches, off-centring, tile-edge options and "
                                         "humidity must agree)");
        }
        if (r != FV3_OK) {
            delete e;
            return fv3::set_error(r, "recording of member " + std::to_string(m) + " failed");
        }
    }
    size_t S = e->rec.sites.size(), bytes = 0;
    e->shape.assign(S, 0);
    e->grid.assign(S, dim3(1, 1, 1));
    e->arg_off.resize(S);
    e->tab_off.resize(S);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (size_t s = 0; s < S; s++) {
            auto it = g_tune_cache.find(e->rec.sites[s].kmulti);
            if (e->rec.sites[s].tunable && it != g_tune_cache.end()) e->shape[s] = it->second;
        }
    }
    for (size_t s = 0; s < S; s++) {
        e->arg_off[s] = bytes;
        bytes += align256(e->rec.sites[s].blob.size());
        e->tab_off[s] = bytes;
        bytes += align256((size_t)members * sizeof(MemberBlk));
    }
    if (hipMalloc((void **)&e->dbuf, bytes) != hipSuccess) {
        delete e;
        return fv3::set_error(FV3_ENOMEM, "ensemble table allocation failed");
    }
    for (size_t s = 0; s < S; s++) {
        const Site &T = e->rec.sites[s];
        if (hipMemcpy(e->dbuf + e->arg_off[s], T.blob.data(), T.blob.size(), hipMemcpyHostToDevice) != hipSuccess ||
            upload_table(e, s) != FV3_OK) {
            fv3_ensemble_free(e);
            return fv3::set_error(FV3_EDEVICE, "ensemble table upload failed");
        }
    }
    if (e->use_graph && hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking) != hipSuccess) {
        fv3_ensemble_free(e);
        return fv3::set_error(FV3_EDEVICE, "stream creation failed");
    }
    *out = e;
    return FV3_OK;
}

fv3_status fv3_ensemble_free(fv3_ensemble *e)
{
    if (!e) return FV3_OK;
    (void)hipDeviceSynchronize();
    drop_graph(e);
    if (e->cap) (void)hipStreamDestroy(e->cap);
    if (e->dbuf) (void)hipFree(e->dbuf);
    delete e;
    return FV3_OK;
}

fv3_status fv3_ensemble_run(fv3_ensemble *e, void *stream)
{
    if (!e) return fv3::set_error(FV3_EINVAL, "NULL ensemble");
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != e->device)
        return fv3::set_error(FV3_EDEVICE, "current HIP device differs from the ensemble's device");
    hipStream_t st = (hipStream_t)stream;
    if (e->use_graph) {
        if (!e->exec) {
            fv3_status r = build_graph(e);
            if (r != FV3_OK) return r;
        }
        if (hipGraphLaunch(e->exec, st) != hipSuccess) return fv3::set_error(FV3_EDEVICE, "graph launch failed");
        return FV3_OK;
    }
    if (launch_call(e, st) != hipSuccess) return fv3::set_error(FV3_EDEVICE, "ensemble launch failed");
    return FV3_OK;
}

fv3_status fv3_ensemble_tune(fv3_ensemble *e, int reps, fv3_tune_report *rep, void *stream)
{
    if (!e || reps < 1) return fv3::set_error(FV3_EINVAL, "NULL ensemble or reps < 1");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return fv3::set_error(FV3_EDEVICE, "event creation failed");
    fv3_tune_report R{};
    auto time_range = [&](size_t lo, size_t hi, float &ms) -> bool {
        if (hipEventRecord(a, st) != hipSuccess) return false;
        for (int r = 0; r < reps; r++)
            if (launch_range(e, lo, hi, st) != hipSuccess) return false;
        if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess) return false;
        return hipEventElapsedTime(&ms, a, b) == hipSuccess;
    };
    const size_t s0 = e->rec.marks[0], s1 = e->rec.marks[1];
    bool ok = true;
    // the substep's time with the shapes in force before tuning
    float before = 0.f;
    ok = ok && launch_range(e, s0, s1, st) == hipSuccess && time_range(s0, s1, before);
    std::map<const void *, int> found;
    for (size_t s = 0; s < e->rec.sites.size() && ok; s++) {
        const Site &S = e->rec.sites[s];
        if (!S.tunable) continue;
        R.tunable_sites++;
        int choice = -1;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(S.kmulti);
            if (it != g_tune_cache.end()) choice = it->second;
        }
        if (choice < 0) {
            auto f = found.find(S.kmulti);
            if (f != found.end()) choice = f->second;
        }
        if (choice >= 0) {
            R.reused++;
        } else {
            float best = 1e30f;
            double t0 = 0.0;
            for (int c = 0; c < kNumShapes && ok; c++) {
                e->shape[s] = c;
                ok = upload_table(e, s) == FV3_OK && launch_site(e, s, st) == hipSuccess;
                float ms = 0.f;
                ok = ok && time_range(s, s + 1, ms);
                t0 += ms;
                if (ok && ms < best) {
                    best = ms;
                    choice = c;
                }
            }
            R.searched++;
            R.search_ms += t0;
            found[S.kmulti] = choice;
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[S.kmulti] = choice;
        }
        e->shape[s] = choice < 0 ? 0 : choice;
        ok = ok && upload_table(e, s) == FV3_OK;
    }
    float after = 0.f;
    ok = ok && time_range(s0, s1, after);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (!ok) return fv3::set_error(FV3_EDEVICE, "tuning launch failed");
    drop_graph(e);
    R.sites = (int)e->rec.sites.size();
    R.substep_ms_before = before / reps;
    R.substep_ms_after = after / reps;
    if (rep) *rep = R;
    return FV3_OK;
}

int fv3_ensemble_shapes(const fv3_ensemble *e, char *names, int names_cap, int *block_x, int *block_y, int cap)
{
    if (!e || !names || !block_x || !block_y) return (int)fv3::set_error(FV3_EINVAL, "NULL argument");
    int k = 0, pos = 0;
    for (size_t s = 0; s < e->rec.sites.size() && k < cap; s++) {
        const Site &S = e->rec.sites[s];
        dim3 b = S.tunable ? kShapes[e->shape[s]] : S.blk;
        int len = (int)S.name.size() + 1;
        if (pos + len > names_cap) break;
        std::copy(S.name.c_str(), S.name.c_str() + len, names + pos);
        pos += len;
        block_x[k] = (int)b.x;
        block_y[k] = (int)b.y;
        k++;
    }
    return k;
}

fv3_status fv3_acoustic_substeps_batched(fv3_state *const *states, const fv3_grid *const *grids, int members,
                                         double dt, int n_split, void *stream)
{
    fv3_ensemble *e = nullptr;
    fv3_status r = fv3_ensemble_create(states, grids, members, dt, n_split, 0, &e);
    if (r != FV3_OK) return r;
    r = fv3_ensemble_run(e, stream);
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess && r == FV3_OK)
        r = fv3::set_error(FV3_EDEVICE, "stream synchronisation failed");
    fv3_ensemble_free(e);
    return r;
}

}  // extern "C"
