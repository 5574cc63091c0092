// bst_internal.h -- plan layout and kernel launchers shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstddef>
#include <vector>

#include "bst.h"

namespace bst {
// Host-side trace range (roctx): shows each entry point and pipeline stage as
// a named range in rocprofv3 --marker-trace; a cheap call when no profiler runs.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};
}  // namespace bst

struct bst_plan_s {
    bst_params prm;      // copy of the caller's parameters (angles pointer cleared)
    int n, V, N;         // detector bins, projections, output side
    int M, G;            // radial FFT length P_r*n, Cartesian grid side P_c*N
    int logM, logG;
    int S;               // row stride of a polar spectrum, complex values: M/2 + 2 (+3 for Keys)
    int lead;            // slots before sample 0 in a polar row: 1 (conj of sample 1) for Keys, else 0
    int taps;            // radial taps of the gather: 2 (linear) or 4 (Keys)
    int GT;              // columns per 8-row tile row of the half-transformed grid: G/2
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
    float2* kc;          // [M/2]        dt * K[m] * A(sigma_m) * exp(2 pi i sigma_m beta dt) of P4
    float2* tw_M;        // [M]          exp(-2 pi i k/M)
    float2* tw_G;        // [G]          exp(-2 pi i k/G)
    double* bf_c;        // [V]          cos(theta_j) * d/dt   (brute force)
    double* bf_s;        // [V]          sin(theta_j) * d/dt
    float* bf_w;         // [V]          w_j
    double2* ang;        // [V]          (cos theta_j, sin theta_j), gather angle residuals
    float* inv_gap;      // [V]          1 / (theta_{j+1} - theta_j), last gap to theta_0 + pi
    // adjoint (bst_project): transposed gather as CSR lists per polar sample
    bool adjoint;
    void* adj_block;
    int* csr_off;        // [V*M/2 + 1]  entry range of polar sample j*M/2 + m
    uint2* csr_ent;      // [entries]    (point index a*G + b | conj << 31, weight bits)
    size_t n_entries;
    float* proj_row;     // [V]          d^2 / (dt w_j): makes R the weighted adjoint of B
    float* mono_phi;     // [n]          phi(t_i - beta dt), monopole Gaussian (if enabled)
    bool f64;            // dtype BST_F64: the FP64 gradient-check path (k_fp64.hip)
    double* taper64;     // [n]          FP64 plans: P1 taper
    double2* kc64;       // [M/2]        FP64 plans: K[m] A(sigma_m) exp(2 pi i sigma_m beta dt)
    double* ramp_h;      // [n]          dt h[d], d = 0..n-1: the band-limited ramp kernel of the
                         //              brute-force comparison (h[d] = h[-d])
    bool monopole;
    float mono_inv, mono_amp, mono_rho_px;
    // tent angular rule: small-radius ("wide") points, column by column
    bool tent;
    size_t tent_w;       // wide point slots (origin slot included)
    int tent_rows;       // radial samples the wide points read: min(M/2, floor(rscale V/pi) + 2)
    size_t tent_chunks;  // tap chunks (at most kTentChunk angle taps each)
    void* tent_block;
    int2* tent_cols;     // [G/2]        (first slot of column a, B_a): rows |b| <= B_a are wide
    int4* tent_chunk;    // [chunks]     (slot, first tap j, last tap j, 0) in the continuation
    int* tent_coff;      // [tent_w + 1] chunk range of each slot
    int gather_slices;   // slices per gather block (coordinates reused across them),
                         // a multiple of kPolarSlices
};

namespace bst {

// record a HIP error for bst_last_error_string (calling thread)
void set_last_error(hipError_t e);
// record a message for bst_last_error_string (calling thread)
void set_last_error_text(const char* text);
// workspace bytes bst_backproject needs for `batch` slices (0 for batch <= 0)
size_t backproject_workspace_need(bst_plan_t plan, int32_t batch);
// bst_backproject with its argument checks, on a given workspace
bst_status backproject_in(bst_plan_t plan, const float* sino, float* img, int32_t batch, void* ws,
                          size_t ws_bytes, void* stream);

struct WsLayout {
    size_t polar_off, dc_off, grid_off, mass_off;
    size_t tent_off, tent_trans_off, tent_part_off, tent_wsum_off;  // tent rule buffers
    size_t total;
};
// Sizes of the tent rule's buffers (all zero without it): wide points W, the
// radius-major copy's rows x V per slice, tap chunks C.
struct TentSizes {
    size_t W = 0, rowsV = 0, C = 0;
};
// slices whose polar spectra are stored interleaved (sample by sample): the
// gather reads both with every tap
constexpr int kPolarSlices = 2;
// Slices per polar group of an ordinary batch: cubic radial taps read four
// samples per row, twice the bytes per slice, and run fastest one slice per
// group (eight 16-byte reads per point otherwise pile up in flight).
constexpr int polar_group(int taps) { return taps == 4 ? 1 : kPolarSlices; }

// Layout of the polar spectra of one group of Q slices, S slots per angle.
// Q = 2: tiles of 2 angles x 4 slots x 2 slices (128 bytes, one cache line),
// ceil(V/2) rows of ceil(S/4) tiles. The four samples (j0, m0..m0+1) x (j0+1,
// m0..m0+1) a linear-tap point reads mostly fall into one or two such lines,
// where rows of single angles spread them over two to four. Q = 1: rows
// [V][S] of single samples.
struct PolarTiles {
    int Q, V, S;
    __host__ __device__ int tiles_per_row() const { return (S + 3) >> 2; }
    // complex values of one group
    __host__ __device__ size_t group_elems() const {
        if (Q == 2) return (size_t)((V + 1) >> 1) * (size_t)tiles_per_row() * 16u;
        return (size_t)V * (size_t)S * (size_t)Q;
    }
    // index (in Q-slice samples, 8 Q bytes) of sample (j, slot) in its group
    __host__ __device__ size_t sample(int j, int slot) const {
        if (Q == 2)
            return ((size_t)(j >> 1) * (size_t)tiles_per_row() + (size_t)(slot >> 2)) * 8u + (size_t)((j & 1) * 4) +
                   (size_t)(slot & 3);
        return (size_t)j * (size_t)S + (size_t)slot;
    }
};
// slices interleaved in the tent rule's radius-major copy
constexpr int kTentSlices = 8;
// slices interleaved in the projector's Cartesian spectra (and summed together
// by one thread of its transposed gather)
constexpr int kProjInterleave = 16;
// Partial sinogram sums per slice for the monopole mass (one per reduction block).
constexpr int kMassChunks = 64;
// Row stride of a polar spectrum and tile-row width of the grid (complex values).
int polar_stride(int M, int interp);
int grid_width(int G);
WsLayout workspace_layout(int n, int V, int N, int M, int G, int batch, int interp, bool monopole,
                          const TentSizes& tent);
// wide points of the tent rule and their column table
size_t tent_columns(int G, int V, std::vector<int2>& cols);
// radial samples the wide points read
int tent_rows(int V, int M, double rscale);
// angle taps per chunk of the tent pre-gather; the chunks of every slot
constexpr int kTentChunk = 32;
void tent_chunks(int V, const std::vector<int2>& cols, std::vector<int4>& chunks, std::vector<int>& coff);

struct ProjWsLayout {
    size_t grid_off, cart8_off, polar_off, total;
};
ProjWsLayout project_workspace_layout(int V, int N, int M, int G, int batch);

struct F64WsLayout {
    size_t polar_off, dc_off, cart_off, polar_t_off, origin_off, total;
};
F64WsLayout f64_workspace_layout(int V, int M, int G, int batch);

struct SpecArgs {
    const float* sino;      // y, or raw counts when flat != nullptr; [batch][V][n]
    const float* const* sino_list;  // or one pointer per slice (device array), if non-null
    const float* flat;      // [batch][n] or nullptr
    const float* dark;      // [batch][n]
    float2* polar;          // groups of Q slices interleaved per sample (PolarTiles)
    float* dc;
    const float* taper;
    const float2* kc;
    const float2* tw;
    int n, V, S;
    int lead;               // slots before sample 0 (1: conj of sample 1 there)
    int tail;               // zero slots after sample M/2 - 1
    float dt;
    // monopole subtraction (mono_part != nullptr): y[i] - m phi[i] is loaded, with
    // m = mono_inv * (sum of the slice's kMassChunks partial sums)
    const float* mono_part; // [batch][kMassChunks]
    const float* mono_phi;  // [n] phi(t_i - beta dt)
    float mono_inv;         // 1 / (V sum_i phi_i)
    // uneven batches: per-slice projection counts (nullptr: V for every slice;
    // else V is the row count of the layout, the largest of them) and the
    // work list of a persistent launch ((group, block) per item; nullptr: the
    // launch grid is the work)
    const int* Vs;
    const int2* items;
    int n_items;
};

struct MassArgs {           // partial sums of each slice's sinogram (monopole mass)
    const float* sino;
    const float* const* sino_list;
    const float* flat;      // raw counts when non-null, as in SpecArgs
    const float* dark;
    float* part;            // [batch][kMassChunks]
    int n, V;
    const int* Vs;          // per-slice projection counts, or nullptr
};

struct GatherArgs {
    const float2* polar;     // groups of Q slices interleaved per sample (PolarTiles)
    const float* dc;
    float2* grid;
    const float2* tw;
    int V, S, N, Mh;
    int GT;                  // grid tile-row width (columns)
    int zero_slot;           // first of the zero slots of a row; also the radius cut-off:
                             // points with r >= zero_slot read only zeros
    int batch, slices_per_block;
    double rscale;
    float vpi_f;             // V / pi
    float dc_scale;
    const double2* ang;      // [V] (cos theta_j, sin theta_j)
    const float* inv_gap;    // [V] 1 / angle gap (non-uniform angles)
    int uniform;             // angles are j pi / V
    // tent angular rule (tent_cols != nullptr): wide points read their value
    // from the pre-gathered patch [batch][tent_w] instead of the polar rows
    const int2* tent_cols;
    const float2* patch;
    int tent_w;
    // uneven batches: per-slice projection counts (nullptr: V for all; else
    // V is the layout's row count), the origin rule's factor (dc_scale =
    // dc_rule / V of the slice), the slices' direction tables (slice s's
    // (cos, sin) of j pi / V_s at ang + ang_off[s]; ang_off nullptr: formed
    // with sincospi) and the work list of a persistent launch ((slice, column
    // block) per item)
    const int* Vs;
    const int* ang_off;
    float dc_rule;
    const int2* items;
    int n_items;
};

struct TentArgs {            // pre-gather of the wide points of the tent rule
    const float2* polar;     // groups of kPolarSlices slices (PolarTiles)
    float2* trans;           // [batch/8][rows][V][8]: the first rows radial samples,
                             // radius-major, 8 slices interleaved
    float2* patch;           // [batch][W]
    float2* part;            // [batch][C] chunk sums (conjugated for the lower half-plane)
    float* wsum;             // [C] chunk weight sums
    const int2* cols;        // [G/2] column table of the wide points
    const int4* chunk;       // [C]
    const int* coff;         // [W + 1]
    int W, C, V, S, lead, rows, ncols;
    double rscale;           // P_r / P_c
};

struct RowArgs {
    const float2* grid;
    float* img;                 // [batch][N][N]
    float* const* img_list;     // or one pointer per slice (device array), if non-null
    const float2* tw;
    int N;
    int GT;                     // grid tile-row width (columns)
    float scale;
    int tiles;                  // row-pair groups per block (set by the launcher)
    // monopole add-back (mono_part != nullptr): + m amp e^-rho I0(rho),
    // rho = rho_px * ((p - N/2)^2 + (q - N/2)^2)
    const float* mono_part;     // [batch][kMassChunks]
    float mono_inv, mono_amp, mono_rho_px;
    // uneven batches: per-slice projection counts for the monopole mass
    // (mono_inv is for V), and the work list of a persistent launch
    // ((slice, block) per item)
    int V;
    const int* Vs;
    const int2* items;
    int n_items;
};

struct F64Args {             // the FP64 gradient-check path (k_fp64.hip)
    const double* sino_in;   // B: sinograms [B][V][n]
    double* sino;            // R: sinograms out (B reads sino_in)
    const double* img_in;    // R: images [B][N][N]
    double* img;             // B: images out
    double2* polar;          // [B][V][M/2 + 2]
    double* dc;              // [B][V]
    double2* cart;           // [B][G][G/2 + 1]
    double2* polar_t;        // [B][V][M/2 + 1]
    double* origin;          // [B]
    const double* taper;     // [n]
    const double2* kc;       // [M/2] K A phase (no dt)
    int n, V, N, M, G;
    double dt, dk2, rscale, dc_rule, row_scale;
};

struct RampArgs {            // the brute-force comparison's ramp filter
    const float* sino;       // [batch][V][n]
    float* out;              // [batch][V][n]
    const double* h;         // [n] dt h[d]
    int n, V;
};

struct BfArgs {
    const float* sino;
    float* img;
    const double* c;
    const double* s;
    const float* w;
    int n, V, N;
};

// adjoint kernels
struct ProjRowArgs {       // image rows -> grid^T tiles
    const float* img;
    float2* grid;
    const float2* tw;      // length G
    int N;
    float scale;           // dk^2
};
struct ProjColArgs {       // grid^T columns -> Cartesian half-plane spectra, interleaved
    const float2* grid;
    float2* cart8;         // [batch/16][G/2 * G][16]
    const float2* tw;
    int N;
    int batch;
    int units;             // blocks: ceil(batch/16) * G/2 (slice group x column)
};
struct ProjGatherArgs {    // CSR transposed gather -> polar^T [V][M/2]
    const float2* cart;    // [batch/16][G/2 * G][16]: the spectra of 16 slices interleaved
    float2* polar;
    const int* off;
    const uint2* ent;
    int samples;           // V * M/2
    int cart_stride;       // G/2 * G complex per slice
    int batch;
    int half_m;            // M/2 radial samples per angle
};
struct ProjPolarArgs {     // polar^T rows -> sinogram rows
    const float2* polar;
    const float2* cart;    // interleaved spectra: slice s's origin value at
                           // cart[(s / 16) * cart_stride * 16 + s % 16]
    float* sino;
    const float* taper;
    const float2* kc;      // dt * K[m] * A * phase (conjugated on use)
    const float2* tw;      // length M
    int n, V, cart_stride;
    float dc_dt;           // dt * dc_scale
    const float* row_scale;  // [V] d^2 / (dt w_j)
};

hipError_t launch_proj_rows(const bst_plan_s& p, const ProjRowArgs& a, int batch, hipStream_t st);
hipError_t launch_proj_cols(const bst_plan_s& p, const ProjColArgs& a, int batch, hipStream_t st);
hipError_t launch_proj_gather(const bst_plan_s& p, const ProjGatherArgs& a, hipStream_t st);
hipError_t launch_proj_polar(const bst_plan_s& p, const ProjPolarArgs& a, int batch, hipStream_t st);

hipError_t launch_mass(const bst_plan_s& p, const MassArgs& a, int batch, hipStream_t st);
hipError_t launch_spectrum(const bst_plan_s& p, const SpecArgs& a, int batch, hipStream_t st);
// Persistent launches of uneven batches: one slice per polar group (no
// interleaving), `blocks` blocks walking the work list in the arguments.
hipError_t launch_spectrum_items(const bst_plan_s& p, const SpecArgs& a, int batch, int blocks, hipStream_t st);
hipError_t launch_gather_items(const bst_plan_s& p, const GatherArgs& a, int blocks, hipStream_t st);
hipError_t launch_row_items(const bst_plan_s& p, const RowArgs& a, int blocks, hipStream_t st);
// blocks per slice and block shape of the stages (for building work lists)
int spectrum_blocks_per_slice(const bst_plan_s& p, int V);  // one-slice groups
int gather_blocks_per_slice(const bst_plan_s& p);
int row_blocks_per_slice(const bst_plan_s& p, int tiles);
int row_max_tiles(const bst_plan_s& p);  // 8-row tiles (4-row past G = 4096) a row block may walk
// copy the interleaved polar spectra out as [batch][V][M/2] complex64 (diagnostics)
hipError_t launch_polar_extract(const bst_plan_s& p, const float2* polar, float2* out, int batch, hipStream_t st);
hipError_t launch_gather_colifft(const bst_plan_s& p, const GatherArgs& a, hipStream_t st);
hipError_t launch_tent(const bst_plan_s& p, const TentArgs& a, int batch, hipStream_t st);
hipError_t launch_row_c2r(const bst_plan_s& p, const RowArgs& a, int batch, hipStream_t st);
hipError_t launch_bruteforce(const bst_plan_s& p, const BfArgs& a, int batch, hipStream_t st);
hipError_t launch_ramp_filter(const bst_plan_s& p, const RampArgs& a, int batch, hipStream_t st);
hipError_t launch_fp64_backproject(const F64Args& a, int batch, hipStream_t st);
hipError_t launch_fp64_project(const F64Args& a, int batch, hipStream_t st);

}  // namespace bst
