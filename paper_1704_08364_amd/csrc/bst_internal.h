// bst_internal.h -- plan layout and kernel launchers shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>

#include "bst.h"

struct bst_plan_s {
    bst_params prm;      // copy of the caller's parameters (angles pointer cleared)
    int n, V, N;         // detector bins, projections, output side
    int M, G;            // radial FFT length P_r*n, Cartesian grid side P_c*N
    int logM, logG;
    int S;               // row stride of a polar spectrum, complex values: M/2 + 2
    bool uniform;        // angles are j*pi/V
    double dt, dk;
    double rscale;       // P_r / P_c: Cartesian index radius -> radial sample index
    double vpi;          // V / pi: angle -> angle index
    float dc_scale;      // origin rule factor divided by V
    float out_scale;     // dk^2
    int device;
    // device tables, one allocation
    void* dev_block;
    float* taper;        // [n]          P1 taper w[i]
    float* kt;           // [M/2]        dt * K[m] of P4
    float2* tw_M;        // [M]          exp(-2 pi i k/M)
    float2* tw_G;        // [G]          exp(-2 pi i k/G)
    double* bf_c;        // [V]          cos(theta_j) * d/dt   (brute force)
    double* bf_s;        // [V]          sin(theta_j) * d/dt
    float* bf_w;         // [V]          w_j
    double2* ang;        // [V]          (cos theta_j, sin theta_j), gather angle residuals
};

namespace bst {

struct WsLayout {
    size_t polar_off, dc_off, grid_off, total;
};
WsLayout workspace_layout(int n, int V, int N, int M, int G, int batch);

struct SpecArgs {
    const float* sino;
    float2* polar;
    float* dc;
    const float* taper;
    const float* kt;
    const float2* tw;
    int n, V, S;
    float dt;
};

struct GatherArgs {
    const float2* polar;
    const float* dc;
    float2* grid;
    const float2* tw;
    int V, S, N, Mh;
    int batch, slices_per_block;
    double rscale;
    float vpi_f;             // V / pi
    float dc_scale;
    const double2* ang;      // [V] (cos theta_j, sin theta_j)
};

struct RowArgs {
    const float2* grid;
    float* img;
    const float2* tw;
    int N;
    float scale;
};

struct BfArgs {
    const float* sino;
    float* img;
    const double* c;
    const double* s;
    const float* w;
    int n, V, N;
};

hipError_t launch_spectrum(const bst_plan_s& p, const SpecArgs& a, int batch, hipStream_t st);
hipError_t launch_gather_colifft(const bst_plan_s& p, const GatherArgs& a, hipStream_t st);
hipError_t launch_row_c2r(const bst_plan_s& p, const RowArgs& a, int batch, hipStream_t st);
hipError_t launch_bruteforce(const bst_plan_s& p, const BfArgs& a, int batch, hipStream_t st);

}  // namespace bst
