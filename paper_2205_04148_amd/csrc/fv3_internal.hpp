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
    M_SIN_U, M_COS_U, M_SIN_V, M_COS_V, M_SIN_A, M_COS_A, M_COUNT,
    // reciprocals (FP64 on the host, then rounded once), so that kernels
    // multiply instead of dividing by a metric term; 0 where the term is 0
    M_RDX = M_COUNT, M_RDY, M_RDXC, M_RDYC, M_RAREA, M_RAREA_C, M_RSIN_U, M_RSIN_V, M_RSIN2_A, M_ALL
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

// A cell next to a tile edge of the cube and its faces on that edge (one, or
// two at a tile corner): our flux (array 0: x-faces, 1: y-faces, in-plane
// offset), the sign with which it enters the cell, and the other tile's copy
// of the face with the sign that maps its flux onto ours.
struct EdgeCell {
    int t, cell, nf;
    int arr[2], off[2], sin[2];
    int pt[2], parr[2], poff[2], spar[2];
};

// Block index handed to a kernel body explicitly (the hardware index when a
// kernel runs alone, the member-local index in an ensemble launch).
struct Bk {
    unsigned x, y, z;
};

// Ensemble launches: per member, its first block in the one-dimensional
// launch grid and its own x/y/z block extents.
struct MemberBlk {
    int b0, gx, gy, gz;
};

// One recorded kernel launch of the substep sequence, for all members:
// the ensemble kernel, the members' argument packs back to back, and per
// member either the point extents and planes (tunable plane kernels, whose
// grid follows the block shape) or the fixed grid dimensions.
struct Site {
    std::string name;
    const void *kmulti = nullptr;
    size_t argsz = 0;
    bool tunable = false;
    dim3 blk;
    std::vector<char> blob;
    std::vector<int> ex, ey, ez;
};

struct Recorder {
    std::vector<Site> sites;
    std::vector<size_t> marks;   // site indices: end of the entry part, end of one substep
    size_t pos = 0, mark = 0;
    int member = 0;
    bool bad = false;
};

}  // namespace fv3

struct fv3_grid {
    fv3_grid_params p;
    fv3::Geo geo;
    int T, n, nz;
    long pitch, rows, lev, off0, pre;
    int bulk_bytes;
    double *met[fv3::M_ALL] = {};             // device, FP64
    float *metf[fv3::M_ALL] = {};             // device, FP32 copies (mixed precision)
    std::vector<double> hmet[fv3::M_ALL];     // host copies
    fv3::Plan planC, planD, planCv, planA;    // scalar, D-grid pair, C-grid pair, cell pair
    fv3::Plan planB;                          // corner (B-grid) scalar
    fv3::EdgeCell *edge_cells = nullptr;      // cube: cells next to tile edges (edge-flux fix-up)
    int edge_count = 0;
    int *flags = nullptr;                     // device error latch [3]: cfl, nonfinite, remap
    double *red = nullptr;                    // device reduction scratch
    long red_elems = 0;
    size_t ws_bytes = 0;
    double da_min = 0.0;                      // smallest corner (dual-cell) area
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
size_t workspace_bytes(const fv3_grid *g);
long reduction_elems(const fv3_grid *g);
void timing_start(const char *filter);
int timing_stop(char *names, int names_cap, double *total_ms, long *counts, int cap);
// a launch bracketed by timing_begin / timing_end (when timing_wanted(name))
// is reported by timing_stop under `name`
struct TimingRec {
    const char *name;
    hipEvent_t a, b;
};
bool timing_wanted(const char *name);
void timing_begin(const char *name, hipStream_t st, TimingRec &r);
void timing_end(hipStream_t st, TimingRec &r);
fv3_status run_substeps(fv3_state *s, const fv3_grid *g, double dt, int n_split, int stop_stage,
                        hipStream_t st);
// record the launch sequence of one substep call (entry, one substep, exit)
// of member rec->member into rec instead of launching it
fv3_status record_substeps(fv3_state *s, const fv3_grid *g, double bdt, Recorder *rec);
fv3_status run_tracer(void *const *q, int nq, fv3_state *s, const fv3_grid *g, int nsplt,
                      hipStream_t st);
fv3_status run_mass_sums(const fv3_grid *g, const void *delp, const void *pt, void *const *q,
                         int nq, double *out, hipStream_t st);
fv3_status run_device_copy(const void *src, void *dst, size_t bytes, hipStream_t st);
// allocation-free variant: scratch in a fixed device array resolved per device
constexpr int FV3_MAX_DEVICES = 64;
fv3_status noalloc_setup(int device);
long noalloc_mass_doubles(const fv3_grid *g);
fv3_status run_mass_sums_noalloc(const fv3_grid *g, const void *delp, const void *pt, void *const *q,
                                 int nq, double *dev_out, hipStream_t st);
fv3_status run_halo_cells(const fv3_grid *g, void *const *f, int nf, int levels, int fp64,
                          hipStream_t st);
// halo of a cell-centred vector (x, y components in tile coordinates)
fv3_status run_halo_pair_cells(const fv3_grid *g, void *fx, void *fy, int levels, int fp64,
                               hipStream_t st);
// remap.hip: vertical remapping of a state to the coordinate ak + bk ps
fv3_status run_remap(fv3_state *s, const fv3_grid *g, const double *ak, const double *bk,
                     void *const *q, int nq, hipStream_t st);

// abi.cpp: record the thread-local message fv3_last_error() returns
fv3_status set_error(fv3_status s, const std::string &msg);
bool device_current(const fv3_grid *g);

}  // namespace fv3
