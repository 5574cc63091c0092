/*
 * bst.h -- C ABI of the BST backprojection library for AMD MI355X (gfx950).
 *
 * The library computes, slice by slice, the low-complexity backprojection of
 * parallel-beam sinograms through the backprojection-slice theorem (Section 2,
 * Eq. 3 of arXiv:1704.08364): for every projection a 1D FFT along the detector
 * axis (steps P1-P4), an interpolation of the polar spectrum onto a Cartesian
 * frequency grid (P5) and a 2D inverse FFT with shift and crop (P6-P8).
 * Plain backprojection (Eq. 2) and filtered backprojection (x = B F y with the
 * |sigma| ramp, Section 1) are both available; in FBP the ramp and the 1/|sigma|
 * of Eq. 3 cancel.
 *
 * Problem statement (Section 1): a slice's sinogram y(t, theta) holds V
 * projections at angles theta_j = j*pi/V in [0, pi), each of n detector bins
 * t_i = (i - n/2)*2/n; the image is N x N with pixel centres
 * u = ((q - N/2)*2/N, (p - N/2)*2/N) for row p, column q.
 *
 * Memory conventions
 *   - Every large buffer (sinograms, images, workspace) is device memory owned
 *     by the caller. A plan owns only small device tables (twiddles, tapers,
 *     weights), freed by bst_destroy.
 *   - sino: float32 [batch][V][n], detector index fastest, contiguous.
 *     img : float32 [batch][N][N], row p = u2, column q = u1, contiguous.
 *   - Input and output buffers must not overlap; the workspace must not
 *     overlap either.
 *   - All compute calls are asynchronous on the given HIP stream (hipStream_t
 *     passed as void*; NULL = the default stream) and return once the kernels
 *     are enqueued. The plan is immutable after creation and may be shared by
 *     host threads; concurrent calls on different streams need separate
 *     workspaces.
 *
 * Errors
 *   - Every function returns a bst_status. Argument errors are detected on the
 *     host before any device work: nothing is enqueued and outputs are untouched.
 *   - BST_E_DEVICE reports a failed HIP runtime call (no GPU, launch failure);
 *     bst_last_error_string() gives the HIP message for the calling thread.
 */
#ifndef BST_H_
#define BST_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bst_plan_s* bst_plan_t;

typedef enum {
    BST_OK = 0,
    BST_E_NULL = 1,         /* a required pointer is NULL                         */
    BST_E_SHAPE = 2,        /* sizes out of range or inconsistent                 */
    BST_E_ANGLES = 3,       /* angles not finite, not increasing or not in [0,pi) */
    BST_E_PARAM = 4,        /* unknown filter / taper / padding value             */
    BST_E_WORKSPACE = 5,    /* workspace smaller than bst_workspace_size          */
    BST_E_NOMEM = 6,        /* device allocation of the plan tables failed        */
    BST_E_DEVICE = 7,       /* a HIP runtime call failed                          */
    BST_E_UNSUPPORTED = 8,  /* valid request the library as compiled lacks       */
    BST_E_BATCH = 9,        /* batch < 0 or batch > max_batch                     */
    BST_E_ALIAS = 10        /* input, output or workspace overlap                 */
} bst_status;

typedef enum {
    BST_FILTER_NONE = 0,    /* plain backprojection b = B y (Eq. 2, via Eq. 3)      */
    BST_FILTER_RAMP = 1     /* filtered backprojection x = B F y, |sigma| ramp     */
} bst_filter;

typedef enum {
    BST_TAPER_DEAPOD = 0,   /* 1/sinc^2(t dsigma): undoes radial linear interpolation */
    BST_TAPER_NONE = 1,
    BST_TAPER_KAISER = 2,   /* Kaiser-Bessel I0(beta sqrt(1-t^2)) / I0(beta)          */
    BST_TAPER_KEYS = 3      /* 1/Khat(t dsigma), Khat(v) = sinc^3(v) (3 sinc(v) - 2 cos(pi v)):
                               undoes radial cubic (Keys) interpolation                */
} bst_taper;

/* Radial interpolation of step P5 (the paper asks for "an interpolation"; the
 * angle direction is always linear). */
typedef enum {
    BST_INTERP_LINEAR = 0,  /* samples m0, m0+1                                       */
    BST_INTERP_KEYS = 1     /* Keys cubic convolution (a = -1/2), samples m0-1 .. m0+2,
                               sample -1 = conj of sample 1; narrows the gap to brute
                               force (pair it with BST_TAPER_KEYS)                    */
} bst_interp;

/* Angular kernel of step P5. */
typedef enum {
    BST_ANGULAR_LINEAR = 0, /* the two bracketing angles, linear weights              */
    BST_ANGULAR_TENT = 1    /* where one Cartesian cell spans several polar angles
                               (radius rho < V/pi grid steps) all angles within
                               h = V/(pi rho) steps, tent weights (1 - |q - j|/h)
                               normalised; elsewhere linear. Uniform angles,
                               BST_INTERP_LINEAR and V/pi < G/2 - 1 only. Its transpose (bst_project)
                               is then a close Radon approximation; the backprojection
                               is as accurate as with LINEAR. Costs a pre-gather
                               kernel over the ~V^2/(2 pi) small-radius points and a
                               [batch][that many] complex64 workspace array        */
} bst_angular;

/* Arithmetic of a plan. BST_F64 plans run plain double-precision kernels on
 * double buffers (bst_backproject_f64, bst_project_f64): a path for checking
 * gradients of least-squares objectives against finite differences and B, R
 * against an FP64 reference, not for speed. They require n_det <= 512,
 * uniform angles, BST_INTERP_LINEAR, BST_ANGULAR_LINEAR and no monopole
 * (BST_E_UNSUPPORTED otherwise); every other parameter applies. */
typedef enum {
    BST_F32 = 0,
    BST_F64 = 1
} bst_dtype;

typedef struct {
    int32_t n_det;          /* n: detector bins; power of two in [16, 4096]            */
    int32_t n_angles;       /* V: projections; [2, 16384]                               */
    int32_t n_out;          /* N: output side; must equal n_det in this version         */
    const double* angles;   /* host, V values, strictly increasing in [0, pi); NULL =
                               uniform j*pi/V. Step P5 brackets each direction in the
                               period-pi continuation of the angle sequence            */
    int32_t pad_radial;     /* P_r in {1,2,4}: FFT length M = P_r*n <= 8192 (P2); 0 -> 2 */
    int32_t pad_cart;       /* P_c in {1,2,4}: Cartesian grid G = P_c*N <= 8192; 0 -> 2  */
    int32_t filter;         /* bst_filter                                                */
    int32_t taper;          /* bst_taper (step P1)                                       */
    double taper_beta;      /* Kaiser-Bessel beta, >= 0                                  */
    int32_t max_batch;      /* largest batch a call may pass; >= 1                       */
    int32_t device;         /* HIP device ordinal the plan's tables live on              */
    int32_t adjoint;        /* nonzero: also build the tables of bst_project (the
                               transposed gather, ~8 bytes per Cartesian-point stencil
                               entry: ~210 MB at N = 2048, P = 2)                       */
    int32_t apodization;    /* bst_apodization: low-pass window A(sigma/sigma_Nyquist)
                               multiplying the radial weight of P4 (the "low-pass
                               filtering" stage F of Section 3)                          */
    double center_shift;    /* known rotation-axis offset beta, detector bins: the data
                               are y(t - beta*dt, theta) (Section 1, "Centering"); P4
                               multiplies by exp(+2 pi i sigma beta dt). |beta| < n/4    */
    int32_t interp;         /* bst_interp (step P5)                                      */
    double monopole_width;  /* BST_FILTER_NONE only; 0 = off. Width s (units of t: the
                               detector spans [-1, 1)) of a unit-mass Gaussian phi on the
                               rotation axis. Against the origin artifacts of Section 2,
                               m phi, m = mean_j sum_i y_ji / sum_i phi(t_i - beta dt), is
                               subtracted from every projection before P1 and its
                               backprojection m (pi/(sqrt(2 pi) s)) e^-rho I0(rho),
                               rho = |u|^2/(4 s^2), added to the image. The 1/|x| mass
                               tail of B y then no longer wraps around the FFT grid.
                               4 dt <= s <= 2; not with adjoint (the result is no longer
                               the transpose of bst_project). Adds a reduction kernel
                               and a [batch][64] float32 workspace array.                */
    int32_t angular;        /* bst_angular (step P5)                                     */
    int32_t dtype;          /* bst_dtype: BST_F32 (default) or BST_F64, the gradient-check
                               path (bst_backproject_f64 / bst_project_f64 only)        */
    int32_t gather_slices;  /* slices each block of the step-P5/P6 gather kernel handles
                               (its interpolation coordinates are computed once for
                               them): 0 = the default (32; 8 with cubic taps on
                               Cartesian grids of G <= 2048), else a positive
                               multiple of 2 up to 1024. Results do not depend on it
                               (tuning and tests only)                                  */
} bst_params;

typedef enum {
    BST_APOD_RAMLAK = 0,    /* A = 1                                  */
    BST_APOD_SHEPP = 1,     /* sin(pi x/2) / (pi x/2)                 */
    BST_APOD_HANN = 2,      /* (1 + cos(pi x)) / 2                    */
    BST_APOD_COSINE = 3     /* cos(pi x/2)                            */
} bst_apodization;

/* Fill *p with the defaults: P_r = P_c = 2, RAMP, de-apodising taper, linear
 * radial interpolation, max_batch 1. */
void bst_params_default(bst_params* p, int32_t n_det, int32_t n_angles, int32_t n_out);

/* Host-only validation of *p (no device call). */
bst_status bst_validate(const bst_params* p);

/* Workspace bytes for `batch` slices (host only, no plan needed).
 * bst_backproject: polar spectra of whole groups of two slices, interleaved
 * sample by sample in tiles of 2 angles x 4 samples, [ceil(batch/2)]
 * [ceil(V/2)][ceil((M/2+2)/4)][2][4][2] complex64 (BST_INTERP_KEYS: one slice
 * per group, rows [batch][V][M/2+5], one leading and two more trailing
 * slots), per-projection
 * DC terms [batch][V] float32, the half-transformed grid [batch][N][G/2]
 * complex64 and, with a monopole width, partial sinogram sums [batch][64]
 * float32. With p->adjoint set, the size also covers bst_project: the grid,
 * the full Cartesian half-plane spectra with 16 slices interleaved per point
 * ([ceil(batch/16)][G/2 * G][16]) and the polar adjoint
 * [batch][V][M/2] (complex64); the larger of the two needs is returned. */
bst_status bst_query_workspace(const bst_params* p, int32_t batch, size_t* bytes);

/* The largest batch Q <= p->max_batch whose device buffers fit in budget_bytes
 * (host only, no plan needed): the sinograms [Q][V][n] and images [Q][N][N]
 * float32 plus the workspace of bst_query_workspace(p, Q). This is the bound
 * the paper puts on its block size Q (Section 4: the per-block allocations of
 * all stages must fit in one GPU's memory). The plan's own tables (a few MB;
 * with adjoint also the transposed-gather lists) come on top. *batch = 0 and
 * BST_E_NOMEM when not even Q = 1 fits. */
bst_status bst_query_max_batch(const bst_params* p, size_t budget_bytes, int32_t* batch);

/* Validate *p, then build the plan on p->device: FP64-derived tables (twiddles
 * of lengths M and G, taper, radial weights K[m] of step P4, angle tables)
 * uploaded in one small allocation. On error *out is left NULL. */
bst_status bst_plan(const bst_params* p, bst_plan_t* out);

/* Same as bst_query_workspace for the plan's own parameters. */
bst_status bst_workspace_size(bst_plan_t plan, int32_t batch, size_t* bytes);

/* BST backprojection of `batch` sinograms (Section 2, steps P0-P8):
 *   BST_FILTER_RAMP: img ~ x = B F y (FBP);  BST_FILTER_NONE: img ~ B y
 *   (a constant sinogram c gives pi*c).
 * sino: device float32 [batch][V][n]; img: device float32 [batch][N][N];
 * ws: device workspace of ws_bytes >= bst_workspace_size(plan, batch).
 * batch == 0 is a no-op. Three kernels are enqueued on `stream` (four with a
 * monopole width: a sinogram-sum kernel first). */
bst_status bst_backproject(bst_plan_t plan, const float* sino, float* img, int32_t batch,
                           void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * bst_backproject, but the workspace is a static device array of the library,
 * 256 MiB on every GPU the library runs on (held from the library's load until
 * the process ends), so the call allocates nothing. The caller passes inputs
 * and outputs as for bst_backproject. Batches whose workspace
 * (bst_workspace_size) exceeds 256 MiB = 268435456 bytes are rejected with
 * BST_E_WORKSPACE before any device work (at N = 2048, P_r = P_c = 2: up to 3
 * slices per call; at N = 1024: up to 15; one slice at N = 4096 needs more). Every call on one GPU uses the same
 * array: calls that overlap in time on one GPU (other streams, other host
 * threads) race and must be serialised by the caller. */
bst_status bst_backproject_noalloc(bst_plan_t plan, const float* sino, float* img, int32_t batch,
                                   void* stream);

/* As bst_backproject, but the input is raw detector counts I [batch][V][n] with
 * per-slice flat (I0) and dark (D) fields [batch][n]; the spectrum kernel forms
 * y = -log((I - D) / (I0 - D)) as it loads (Section 1, "Normalization").
 * Requires I > D and I0 > D; other values give non-finite results. */
bst_status bst_backproject_counts(bst_plan_t plan, const float* counts, const float* flat, const float* dark,
                                  float* img, int32_t batch, void* ws, size_t ws_bytes, void* stream);

/* As bst_backproject, and records 4 caller-created HIP events (hipEvent_t
 * passed as void*) on `stream`: before the spectrum kernel, between the
 * kernels, and after the last one, so per-kernel time is measurable. */
bst_status bst_backproject_timed(bst_plan_t plan, const float* sino, float* img, int32_t batch,
                                 void* ws, size_t ws_bytes, void* stream, void* const* events4);

/* Brute-force ("slant-stack") backprojection, Eq. 2 summed directly over the V
 * angles with linear interpolation along t (Section 2, last paragraph):
 *   img[p][q] = sum_j w_j * lerp(sino_j, (u.xi_j)/dt + n/2),  zero outside [0,n).
 * It applies no filter: for FBP pass a ramp-filtered sinogram. Uses the plan's
 * angles (uniform or not) and weights w_j (pi/V, or half the neighbour gap). */
bst_status bst_backproject_bruteforce(bst_plan_t plan, const float* sino, float* img,
                                      int32_t batch, void* stream);

/* FP64 gradient-check path (plans with dtype BST_F64; float entry points
 * return BST_E_UNSUPPORTED for them, and these for BST_F32 plans): the same
 * operators as bst_backproject and bst_project, in double precision,
 * sino double [batch][V][n], img double [batch][N][N], workspace of
 * bst_workspace_size bytes. B: steps P1-P8 of Section 2 with the plan's
 * filter, taper, paddings, apodisation and centre shift; R: its exact adjoint
 * under the weighted inner products (<R f, g> = <f, B g>, as bst_project).
 * bst_project_f64 needs no adjoint tables (its transposed gather adds with
 * FP64 atomics, so its last bits may vary between runs). */
bst_status bst_backproject_f64(bst_plan_t plan, const double* sino, double* img, int32_t batch, void* ws,
                               size_t ws_bytes, void* stream);
bst_status bst_project_f64(bst_plan_t plan, const double* img, double* sino, int32_t batch, void* ws,
                           size_t ws_bytes, void* stream);

/* Ramp filter of the brute-force FBP (the comparison's x = B F y, Section 1):
 * the paper gives no discrete ramp, so this is the band-limited spatial kernel
 * of Kak and Slaney sampled at the detector pitch, h[0] = 1/(4 dt^2),
 * h[d odd] = -1/(pi^2 d^2 dt^2), h[d even] = 0, applied along each projection
 * as a linear (not circular) convolution q[i] = dt sum_k h[i - k] y[k]
 * (FP64 sums). sino, out: device float32 [batch][V][n], not overlapping.
 * Feed `out` to bst_backproject_bruteforce for the brute-force FBP. */
bst_status bst_ramp_filter(bst_plan_t plan, const float* sino, float* out, int32_t batch, void* stream);

/* Projector R, the exact adjoint of bst_backproject: steps P8..P1 of Section 2
 * transposed one by one (crop -> zero-embed, C2R inverse FFT -> forward FFT,
 * gather (linear or cubic radial taps, any angle set) -> the same weights
 * scattered back, 1D FFT -> its transpose, pad -> crop, taper -> taper), scaled
 * so that under the weighted inner products <f,f'> = d^2 sum f f' and
 * <g,g'> = dt sum_j w_j sum_i g g' (w_j = pi/V, or half the neighbour gap)
 *     <R f, g> = <f, B g>   (B = R* as in Section 1).
 * With a BST_FILTER_NONE plan R is a Fourier-slice (Eq. 1) projector; its
 * transposed gridding is exact as an adjoint but, with BST_ANGULAR_LINEAR and
 * where polar samples are denser than Cartesian ones (radius < V/pi grid
 * steps), it weights lattice-aligned angles unevenly, so as a stand-alone Radon
 * approximation it is coarse at low frequencies (several times the signal);
 * with BST_ANGULAR_TENT it is within about 8 % of the Radon transform of a
 * smooth object. img: device float32 [batch][N][N]; sino: device float32
 * [batch][V][n]. Needs a plan built with adjoint != 0 (else BST_E_UNSUPPORTED)
 * and a workspace of bst_workspace_size bytes. Deterministic (no atomics). */
bst_status bst_project(bst_plan_t plan, const float* img, float* sino, int32_t batch,
                       void* ws, size_t ws_bytes, void* stream);

/* Diagnostic: run steps P1-P4 only and copy the polar spectrum
 * (complex64 [batch][V][M/2], Yh_j[m] = dt * K[m] * sum_k z_j[k] e^{-2 pi i k m/M})
 * and the DC terms (float32 [batch][V], dt * sum_i w_i y_j[i]) to caller buffers. */
bst_status bst_debug_spectrum(bst_plan_t plan, const float* sino, void* spec, float* dc,
                              int32_t batch, void* ws, size_t ws_bytes, void* stream);

/* ---- Uneven-size batches (Section 3's pipeline processes blocks of Q
 * sinograms; Section 4 measures its time against Q) ---------------------------
 * Many sinograms of different sizes (n_det[i], n_angles[i]) in one graph
 * launch; every other parameter comes from *base (uniform angles only, FP32;
 * otherwise BST_E_UNSUPPORTED, and per-instance validation as for
 * bst_validate). Instances of equal n form a size class with one plan (built
 * for the class's largest V) and one workspace region; per stage, one
 * persistent kernel per class walks a device work list of (instance, tile)
 * items, each instance with its own V. With the tent angular rule the
 * classes are instead those of equal (n, V), run by the ordinary kernels.
 * Classes run concurrently. Sinograms and images live in two packed device
 * buffers at the element offsets sino_off[i] and img_off[i] (host arrays of
 * `count`), each instance float32 [V_i][n_i] and [n_i][n_i]. The first
 * bst_batch_backproject with a given workspace captures all launches into a
 * hipGraph; later calls only upload the pointer lists and replay it. Calls on
 * one batch must not overlap in time (they share the pointer lists). Results
 * equal bst_backproject's for each instance to rounding. bst_batch_create
 * returns BST_E_BATCH for count < 1 or a size class whose instances have more
 * than 2^31 - 1 angles in total.
 */
typedef struct bst_batch_s* bst_batch_t;

bst_status bst_batch_create(const bst_params* base, int32_t count, const int32_t* n_det,
                            const int32_t* n_angles, bst_batch_t* out);
bst_status bst_batch_workspace_size(bst_batch_t b, size_t* bytes);
bst_status bst_batch_classes(bst_batch_t b, int32_t* n_classes);
/* Autotuner: for every size class, on these inputs, time each stage's
 * persistent grid (1, 2, 4 or 8 blocks per compute unit) and the row stage's
 * tiles per work item (1, 2, 4, 8 or 16 eight-row tiles), keep the fastest,
 * and drop any captured graph. Results do not depend on the choice.
 * Synchronizes the stream. Outputs are overwritten. */
bst_status bst_batch_tune(bst_batch_t b, const float* sinos, const int64_t* sino_off, float* imgs,
                          const int64_t* img_off, void* ws, size_t ws_bytes, void* stream);
bst_status bst_batch_backproject(bst_batch_t b, const float* sinos, const int64_t* sino_off, float* imgs,
                                 const int64_t* img_off, void* ws, size_t ws_bytes, void* stream);
bst_status bst_batch_destroy(bst_batch_t b);

/* Free the plan's device tables and the plan. NULL is accepted. */
bst_status bst_destroy(bst_plan_t plan);

/* Static text for a status code (a bst_status value; any other integer gives
   "unknown status"). */
const char* bst_status_string(int32_t status);

/* Index checks of the checked build (compiled with BST_CHECKED, e.g. by
 * `python -m paper_1704_08364_amd.build --checked`): *flags receives the bits
 * of every kernel index check that failed since the last call (spectrum
 * bits 0-7, gather 8-15, row 16-23, projector 24-31) and they are cleared; a
 * failing index was replaced by 0, so the access stayed in bounds. Device
 * `device`. Returns BST_E_UNSUPPORTED in ordinary builds. */
bst_status bst_debug_check(int32_t device, uint32_t* flags);

/* Text of the last HIP error seen by this thread ("" if none). */
const char* bst_last_error_string(void);

/* Helpers for callers that have no HIP bindings of their own. */
bst_status bst_event_create(void** ev);
bst_status bst_event_destroy(void* ev);
bst_status bst_event_elapsed_ms(void* start, void* stop, float* ms);
bst_status bst_stream_synchronize(void* stream);

#ifdef __cplusplus
}
#endif

#endif /* BST_H_ */
