// Internal declarations of the FV3 acoustic-substep library (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fv3.h"

namespace fv3 {

constexpr int HALO = 3;

// physical constants of the dry system
constexpr double GRAV = 9.80665;
constexpr double RDGAS = 287.05;
constexpr double CP_AIR = 1004.6;
constexpr double P_REF = 1.0e5;

enum Stag { SC = 0, SX = 1, SY = 2, SB = 3 };
enum Metric {
    M_DX = 0, M_DY, M_DXC, M_DYC, M_DXA, M_DYA, M_AREA, M_AREA_C, M_FC, M_FB,
    M_SIN_U, M_COS_U, M_SIN_V, M_COS_V, M_SIN_A, M_COS_A, M_COUNT
};

// Field geometry handed to kernels by value.
struct Geo {
    int n, nz, T;
    int cube;          // 1 on the cubed sphere (corner blocks are views), 0 periodic
    long pitch, lev, off0;
};

// One halo copy: destination and source (tile, in-plane index); `sel` bit 0:
// source is the y component of a pair, bit 1: negate, bit 2: destination is
// the y component.
struct HaloEnt {
    int dt, di, st, si, sel;
};

struct Plan {
    HaloEnt *d = nullptr;
    int count = 0;
};

}  // namespace fv3

struct fv3_grid {
    fv3_grid_params p;
    fv3::Geo geo;
    int T, n, nz;
    long pitch, rows, lev, off0, pre;
    int bulk_bytes;
    double *met[fv3::M_COUNT] = {};           // device, FP64
    float *metf[fv3::M_COUNT] = {};           // device, FP32 copies (mixed precision)
    std::vector<double> hmet[fv3::M_COUNT];   // host copies
    fv3::Plan planC, planD, planCv;           // scalar, D-grid pair, C-grid pair
    int *flags = nullptr;                     // device error latch [2]: cfl, nonfinite
    double *red = nullptr;                    // device reduction scratch
    long red_elems = 0;
    size_t ws_bytes = 0;
};

namespace fv3 {

inline long alloc_elems(const fv3_grid *g, int levels)
{
    return g->off0 - HALO * (g->pitch + 1) + (long)g->T * levels * g->lev + g->pitch;
}

// grid.cpp
fv3_status build_grid(const fv3_grid_params *p, fv3_grid *g, std::string &err);
fv3_status host_metric(const fv3_grid_params *p, int m, double *out, long cap, std::string &err);

// Kernel launchers (kernels.hip).  All take the grid, device pointers and a stream.
struct Work;   // workspace carve-up, defined in kernels.hip
size_t workspace_bytes(const fv3_grid *g);
long reduction_elems(const fv3_grid *g);
void timing_start(const char *filter);
int timing_stop(char *names, int names_cap, double *total_ms, long *counts, int cap);
fv3_status run_substeps(fv3_state *s, const fv3_grid *g, double dt, int n_split, int stop_stage,
                        hipStream_t st);
fv3_status run_tracer(void *const *q, int nq, fv3_state *s, const fv3_grid *g, int nsplt,
                      hipStream_t st);
fv3_status run_mass_sums(const fv3_grid *g, const void *delp, const void *pt, void *const *q,
                         int nq, double *out, hipStream_t st);
fv3_status run_halo_cells(const fv3_grid *g, void *const *f, int nf, int levels, int fp64,
                          hipStream_t st);

}  // namespace fv3
