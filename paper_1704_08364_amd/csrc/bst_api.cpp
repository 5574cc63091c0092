// bst_api.cpp -- the C ABI declared in include/bst.h: host-side validation,
// FP64 plan tables, workspace carving and kernel enqueueing.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "bst_internal.h"

// slices per gather block: the interpolation coordinates are computed once per
// block, so more slices amortise them; cubic taps on grids up to 2048 (one
// slice per polar group, two blocks per compute unit) gain more from a grid of
// more, shorter blocks (N = 2048 at P_c = 1: gather 1.37 ms with 32 slices,
// 1.30 ms with 8)
#ifndef BST_GATHER_SLICES
#define BST_GATHER_SLICES 32
#endif
#ifndef BST_GATHER_SLICES_CUBIC_SMALL
#define BST_GATHER_SLICES_CUBIC_SMALL 8
#endif

namespace bst {
#ifdef BST_CHECKED
unsigned check_flags_spectrum();
unsigned check_flags_gather();
unsigned check_flags_row();
unsigned check_flags_project();
#endif
bool build_adjoint_tables(int V, int M, int G, double rscale, const std::vector<double>& theta, bool uniform,
                          int taps, const std::vector<int2>* tent_cols, std::vector<int>& off,
                          std::vector<uint2>& ent);
}

namespace {

thread_local std::string g_last_error;

bst_status device_fail(hipError_t e) {
    g_last_error = hipGetErrorString(e);
    return BST_E_DEVICE;
}

bool is_pow2(int32_t x) { return x > 0 && (x & (x - 1)) == 0; }

int ilog2(int32_t x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

int pad_or_default(int32_t v) { return v == 0 ? 2 : v; }

// I0(x) = sum_k (x^2/4)^k / (k!)^2; terms fall below 1e-17 of the sum within
// a few dozen steps for the betas a Kaiser-Bessel taper uses.
double bessel_i0(double x) {
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

struct Range {
    uintptr_t lo, hi;
};
bool overlap(Range a, Range b) { return a.lo < b.hi && b.lo < a.hi; }

// RAII guard that makes the plan's device current and restores the caller's.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

namespace bst {

void set_last_error(hipError_t e) { g_last_error = hipGetErrorString(e); }

// Row strides of the polar spectra and of the grid's tile rows. Padding them
// to odd multiples of 256 bytes (to spread rows over memory channels) was
// measured on MI355X: it speeds the spectrum kernel by 7% but slows the
// gather by 4%, a net loss, so both stay unpadded.
// Keys rows: [conj Yh[1], Yh[0 .. M/2-1], four zeros], linear rows: [Yh[0 .. M/2-1], two zeros]
int polar_stride(int M, int interp) { return M / 2 + (interp == BST_INTERP_KEYS ? 5 : 2); }
int grid_width(int G) { return G / 2; }

WsLayout workspace_layout(int n, int V, int N, int M, int G, int batch, int interp, bool monopole,
                          const TentSizes& tent) {
    (void)n;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    WsLayout L{};
    const size_t B = (size_t)batch;
    L.polar_off = 0;
    // whole groups of interleaved slices
    const int Q = polar_group(interp == BST_INTERP_KEYS ? 4 : 2);
    const size_t pgroups = (B + Q - 1) / Q;
    const size_t polar = pgroups * PolarTiles{Q, V, polar_stride(M, interp)}.group_elems() * sizeof(float2);
    L.dc_off = up(L.polar_off + polar);
    const size_t dc = B * (size_t)V * sizeof(float);
    L.grid_off = up(L.dc_off + dc);
    const size_t grid = B * (size_t)N * (size_t)grid_width(G) * sizeof(float2);
    L.mass_off = up(L.grid_off + grid);
    const size_t mass = monopole ? B * (size_t)kMassChunks * sizeof(float) : 0;
    L.tent_off = up(L.mass_off + mass);
    // tent rule: wide-point values [B][W], the radius-major copy [ceil(B/8)][rows][V][8],
    // chunk sums [B][C], chunk weight sums [C] (float)
    const size_t groups = (B + kTentSlices - 1) / kTentSlices;
    L.tent_trans_off = up(L.tent_off + B * tent.W * sizeof(float2));
    L.tent_part_off = up(L.tent_trans_off + groups * kTentSlices * tent.rowsV * sizeof(float2));
    L.tent_wsum_off = up(L.tent_part_off + B * tent.C * sizeof(float2));
    L.total = up(L.tent_wsum_off + tent.C * sizeof(float));
    return L;
}

ProjWsLayout project_workspace_layout(int V, int N, int M, int G, int batch) {
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    ProjWsLayout L{};
    const size_t B = (size_t)batch;
    const size_t plane = (size_t)(G / 2) * (size_t)G;
    const size_t groups = (B + kProjInterleave - 1) / kProjInterleave;
    L.grid_off = 0;
    L.cart8_off = up(B * (size_t)N * (size_t)(G / 2) * sizeof(float2));
    L.polar_off = up(L.cart8_off + groups * kProjInterleave * plane * sizeof(float2));
    L.total = up(L.polar_off + B * (size_t)V * (size_t)(M / 2) * sizeof(float2));
    return L;
}

F64WsLayout f64_workspace_layout(int V, int M, int G, int batch) {
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    F64WsLayout L{};
    const size_t B = (size_t)batch;
    L.polar_off = 0;
    L.dc_off = up(B * (size_t)V * (size_t)(M / 2 + 2) * 16);
    L.cart_off = up(L.dc_off + B * (size_t)V * 8);
    L.polar_t_off = up(L.cart_off + B * (size_t)G * (size_t)(G / 2 + 1) * 16);
    L.origin_off = up(L.polar_t_off + B * (size_t)V * (size_t)(M / 2 + 1) * 16);
    L.total = up(L.origin_off + B * 8);
    return L;
}

size_t workspace_bytes(int n, int V, int N, int M, int G, int batch, bool adjoint, int interp, bool monopole,
                       const TentSizes& tent, bool f64) {
    if (batch == 0) return 0;
    if (f64) return f64_workspace_layout(V, M, G, batch).total;
    size_t need = workspace_layout(n, V, N, M, G, batch, interp, monopole, tent).total;
    if (adjoint) {
        const size_t pj = project_workspace_layout(V, N, M, G, batch).total;
        if (pj > need) need = pj;
    }
    return need;
}

}  // namespace bst

extern "C" {

void bst_params_default(bst_params* p, int32_t n_det, int32_t n_angles, int32_t n_out) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->n_det = n_det;
    p->n_angles = n_angles;
    p->n_out = n_out;
    p->angles = nullptr;
    p->pad_radial = 2;
    p->pad_cart = 2;
    p->filter = BST_FILTER_RAMP;
    p->taper = BST_TAPER_DEAPOD;
    p->taper_beta = 8.0;
    p->max_batch = 1;
    p->device = 0;
    p->adjoint = 0;
    p->apodization = BST_APOD_RAMLAK;
    p->center_shift = 0.0;
    p->interp = BST_INTERP_LINEAR;
    p->monopole_width = 0.0;
    p->angular = BST_ANGULAR_LINEAR;
    p->gather_slices = 0;
    p->dtype = BST_F32;
}

bst_status bst_validate(const bst_params* p) {
    if (!p) return BST_E_NULL;
    if (!is_pow2(p->n_det) || p->n_det < 16 || p->n_det > 4096) return BST_E_SHAPE;
    if (p->n_out != p->n_det) return BST_E_SHAPE;
    if (p->n_angles < 2 || p->n_angles > 16384) return BST_E_SHAPE;
    const int pr = pad_or_default(p->pad_radial), pc = pad_or_default(p->pad_cart);
    if (!(pr == 1 || pr == 2 || pr == 4) || !(pc == 1 || pc == 2 || pc == 4)) return BST_E_PARAM;
    if ((int64_t)pr * p->n_det > 8192 || (int64_t)pc * p->n_out > 8192) return BST_E_SHAPE;
    if (p->filter != BST_FILTER_NONE && p->filter != BST_FILTER_RAMP) return BST_E_PARAM;
    if (p->taper != BST_TAPER_DEAPOD && p->taper != BST_TAPER_NONE && p->taper != BST_TAPER_KAISER &&
        p->taper != BST_TAPER_KEYS)
        return BST_E_PARAM;
    if (p->interp != BST_INTERP_LINEAR && p->interp != BST_INTERP_KEYS) return BST_E_PARAM;

    if (p->taper == BST_TAPER_KAISER && !(std::isfinite(p->taper_beta) && p->taper_beta >= 0.0 &&
                                          p->taper_beta <= 700.0))
        return BST_E_PARAM;
    if (p->apodization < BST_APOD_RAMLAK || p->apodization > BST_APOD_COSINE) return BST_E_PARAM;
    if (!std::isfinite(p->center_shift) || std::fabs(p->center_shift) >= 0.25 * p->n_det) return BST_E_PARAM;
    if (p->angular != BST_ANGULAR_LINEAR && p->angular != BST_ANGULAR_TENT) return BST_E_PARAM;
    if (p->angular == BST_ANGULAR_TENT) {
        if (p->angles || p->interp != BST_INTERP_LINEAR) return BST_E_PARAM;
        // the wide disk (radius V/pi) must stay inside the Cartesian grid
        if ((double)p->n_angles / M_PI >= (double)(pc * p->n_out / 2 - 1)) return BST_E_PARAM;
    }
    if (p->monopole_width != 0.0) {
        // plain B only, not with the adjoint, and a Gaussian the detector resolves
        const double s = p->monopole_width, dt = 2.0 / p->n_det;
        if (!std::isfinite(s) || s < 4.0 * dt || s > 2.0) return BST_E_PARAM;
        if (p->filter != BST_FILTER_NONE || p->adjoint) return BST_E_PARAM;
    }
    if (p->max_batch < 1) return BST_E_BATCH;
    if (p->device < 0) return BST_E_PARAM;
    if (p->gather_slices < 0 || p->gather_slices > 1024 || p->gather_slices % bst::kPolarSlices != 0)
        return BST_E_PARAM;
    if (p->dtype != BST_F32 && p->dtype != BST_F64) return BST_E_PARAM;
    if (p->dtype == BST_F64 && (p->n_det > 512 || p->angles || p->interp != BST_INTERP_LINEAR ||
                                p->angular != BST_ANGULAR_LINEAR || p->monopole_width != 0.0))
        return BST_E_UNSUPPORTED;
    if (p->angles) {
        double prev = -1.0;
        for (int j = 0; j < p->n_angles; ++j) {
            const double a = p->angles[j];
            if (!std::isfinite(a) || a < 0.0 || a >= M_PI || a <= prev) return BST_E_ANGLES;
            prev = a;
        }
    }
    return BST_OK;
}

namespace {
// complex values per slice of the tent rule's buffers: the wide points'
// values and the radius-major copy of the polar samples they read
bst::TentSizes params_tent_sizes(const bst_params* p, int M, int G) {
    bst::TentSizes t;
    if (p->angular != BST_ANGULAR_TENT) return t;
    std::vector<int2> cols;
    std::vector<int4> chunks;
    std::vector<int> coff;
    const double rscale = (double)pad_or_default(p->pad_radial) / (double)pad_or_default(p->pad_cart);
    t.W = bst::tent_columns(G, p->n_angles, cols);
    bst::tent_chunks(p->n_angles, cols, chunks, coff);
    t.rowsV = (size_t)bst::tent_rows(p->n_angles, M, rscale) * (size_t)p->n_angles;
    t.C = chunks.size();
    return t;
}

bst::TentSizes tent_sizes(const bst_plan_s* plan) {
    bst::TentSizes t;
    if (!plan->tent) return t;
    t.W = plan->tent_w;
    t.rowsV = (size_t)plan->tent_rows * (size_t)plan->V;
    t.C = plan->tent_chunks;
    return t;
}
}  // namespace

bst_status bst_query_workspace(const bst_params* p, int32_t batch, size_t* bytes) {
    if (!bytes) return BST_E_NULL;
    const bst_status st = bst_validate(p);
    if (st != BST_OK) return st;
    if (batch < 0 || batch > p->max_batch) return BST_E_BATCH;
    const int M = pad_or_default(p->pad_radial) * p->n_det;
    const int G = pad_or_default(p->pad_cart) * p->n_out;
    *bytes = bst::workspace_bytes(p->n_det, p->n_angles, p->n_out, M, G, batch, p->adjoint != 0, p->interp,
                                  p->monopole_width != 0.0, params_tent_sizes(p, M, G), p->dtype == BST_F64);
    return BST_OK;
}

bst_status bst_query_max_batch(const bst_params* p, size_t budget_bytes, int32_t* batch) {
    if (!batch) return BST_E_NULL;
    *batch = 0;
    const bst_status st = bst_validate(p);
    if (st != BST_OK) return st;
    const int M = pad_or_default(p->pad_radial) * p->n_det;
    const int G = pad_or_default(p->pad_cart) * p->n_out;
    const size_t io = ((size_t)p->n_angles * p->n_det + (size_t)p->n_out * p->n_out) * sizeof(float);
    const bst::TentSizes tw = params_tent_sizes(p, M, G);
    auto need = [&](int32_t q) {
        return (size_t)q * io * (p->dtype == BST_F64 ? 2 : 1) +
               bst::workspace_bytes(p->n_det, p->n_angles, p->n_out, M, G, q, p->adjoint != 0, p->interp,
                                    p->monopole_width != 0.0, tw, p->dtype == BST_F64);
    };
    // need(q) grows with q: binary search for the last q that fits
    int32_t lo = 0, hi = p->max_batch;
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo + 1) / 2;
        if (need(mid) <= budget_bytes) lo = mid;
        else hi = mid - 1;
    }
    *batch = lo;
    return lo > 0 ? BST_OK : BST_E_NOMEM;
}

bst_status bst_plan(const bst_params* p, bst_plan_t* out) {
    if (!out) return BST_E_NULL;
    *out = nullptr;
    const bst_status st = bst_validate(p);
    if (st != BST_OK) return st;

    bst_plan_s* pl = new (std::nothrow) bst_plan_s();
    if (!pl) return BST_E_NOMEM;
    pl->prm = *p;
    pl->prm.angles = nullptr;
    pl->prm.pad_radial = pad_or_default(p->pad_radial);
    pl->prm.pad_cart = pad_or_default(p->pad_cart);
    pl->n = p->n_det;
    pl->V = p->n_angles;
    pl->N = p->n_out;
    pl->M = pl->prm.pad_radial * pl->n;
    pl->G = pl->prm.pad_cart * pl->N;
    pl->logM = ilog2(pl->M);
    pl->logG = ilog2(pl->G);
    pl->S = bst::polar_stride(pl->M, p->interp);
    pl->lead = (p->interp == BST_INTERP_KEYS) ? 1 : 0;
    pl->taps = (p->interp == BST_INTERP_KEYS) ? 4 : 2;
    pl->GT = bst::grid_width(pl->G);
    pl->uniform = (p->angles == nullptr);
    pl->dt = 2.0 / pl->n;
    const double d = 2.0 / pl->N;
    pl->dk = 1.0 / (pl->G * d);
    pl->rscale = (double)pl->prm.pad_radial / (double)pl->prm.pad_cart;
    pl->vpi = (double)pl->V / M_PI;
    const double kappa = 4.0 * std::asinh(1.0);
    const double dc_rule = (p->filter == BST_FILTER_RAMP) ? 1.0 : kappa / pl->dk;
    pl->dc_scale = (float)(dc_rule / pl->V);
    pl->out_scale = (float)(pl->dk * pl->dk);
    pl->device = p->device;
    pl->adjoint = (p->adjoint != 0);
    pl->gather_slices = p->gather_slices > 0
                            ? p->gather_slices
                            : ((pl->taps == 4 && pl->G <= 2048) ? BST_GATHER_SLICES_CUBIC_SMALL : BST_GATHER_SLICES);
    pl->monopole = (p->monopole_width != 0.0);
    pl->tent = (p->angular == BST_ANGULAR_TENT);
    pl->f64 = (p->dtype == BST_F64);

    // ---- FP64 tables ----
    const int n = pl->n, M = pl->M, G = pl->G, V = pl->V;
    const double dsig = 1.0 / (M * pl->dt);
    std::vector<float> taper(n), bf_w(V);
    std::vector<double> taper64(n);
    std::vector<double2> kc64(M / 2);
    std::vector<float2> kc(M / 2);
    std::vector<float2> twM(M), twG(G);
    std::vector<double> bf_c(V), bf_s(V), theta(V);
    std::vector<double2> ang(V);
    std::vector<float> inv_gap(V), proj_row(V);
    for (int i = 0; i < n; ++i) {
        const double t = (i - n / 2) * pl->dt;
        double w = 1.0;
        if (p->taper == BST_TAPER_DEAPOD) {
            const double x = M_PI * t * dsig;
            const double sc = (x == 0.0) ? 1.0 : std::sin(x) / x;
            w = 1.0 / (sc * sc);
        } else if (p->taper == BST_TAPER_KEYS) {
            // transform of the Keys kernel (a = -1/2): sinc^3 (3 sinc - 2 cos), by
            // integrating its two cubic pieces against cos(2 pi v x)
            const double x = M_PI * t * dsig;
            const double sc = (x == 0.0) ? 1.0 : std::sin(x) / x;
            w = 1.0 / (sc * sc * sc * (3.0 * sc - 2.0 * std::cos(x)));
        } else if (p->taper == BST_TAPER_KAISER) {
            const double arg = 1.0 - t * t;
            w = bessel_i0(p->taper_beta * std::sqrt(arg > 0.0 ? arg : 0.0)) / bessel_i0(p->taper_beta);
        }
        taper[i] = (float)w;
        taper64[i] = w;
    }
    for (int m = 0; m < M / 2; ++m) {
        double K;
        if (p->filter == BST_FILTER_RAMP) K = 1.0;
        else K = (m == 0) ? 0.0 : (M * pl->dt) / (double)m;
        const double x = 2.0 * m / (double)M;  // sigma_m / sigma_Nyquist
        double A = 1.0;
        if (p->apodization == BST_APOD_SHEPP) A = (x == 0.0) ? 1.0 : std::sin(M_PI * x / 2) / (M_PI * x / 2);
        else if (p->apodization == BST_APOD_HANN) A = 0.5 * (1.0 + std::cos(M_PI * x));
        else if (p->apodization == BST_APOD_COSINE) A = std::cos(M_PI * x / 2);
        const double ph = 2.0 * M_PI * (double)m * p->center_shift / (double)M;
        const double wr = pl->dt * K * A;
        kc[m] = make_float2((float)(wr * std::cos(ph)), (float)(wr * std::sin(ph)));
        kc64[m] = make_double2(K * A * std::cos(ph), K * A * std::sin(ph));
    }
    for (int k = 0; k < M; ++k) {
        const double a = -2.0 * M_PI * (double)k / (double)M;
        twM[k] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    for (int k = 0; k < G; ++k) {
        const double a = -2.0 * M_PI * (double)k / (double)G;
        twG[k] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    for (int j = 0; j < V; ++j) theta[j] = p->angles ? p->angles[j] : (double)j * M_PI / (double)V;
    const double ratio = d / pl->dt;
    for (int j = 0; j < V; ++j) ang[j] = make_double2(std::cos(theta[j]), std::sin(theta[j]));
    // 1 / (theta_{j+1} - theta_j) in the period-pi continuation (the last gap wraps to theta_0 + pi)
    for (int j = 0; j < V; ++j) {
        const double next = (j == V - 1) ? theta[0] + M_PI : theta[j + 1];
        inv_gap[j] = (float)(1.0 / (next - theta[j]));
    }
    for (int j = 0; j < V; ++j) {
        bf_c[j] = std::cos(theta[j]) * ratio;
        bf_s[j] = std::sin(theta[j]) * ratio;
        double w;
        if (pl->uniform) {
            w = M_PI / V;
        } else {
            const double prev = (j == 0) ? theta[V - 1] - M_PI : theta[j - 1];
            const double next = (j == V - 1) ? theta[0] + M_PI : theta[j + 1];
            w = 0.5 * (next - prev);
        }
        bf_w[j] = (float)w;
        proj_row[j] = (float)(d * d / (pl->dt * w));
    }

    // monopole: phi(t_i - beta dt) = exp(-(t_i - beta dt)^2 / (2 s^2)) / (sqrt(2 pi) s); the
    // add-back m (pi / (sqrt(2 pi) s)) e^-rho I0(rho), rho = |u|^2 / (4 s^2) = rho_px * pixels^2
    std::vector<float> mono_phi(n, 0.0f);
    if (pl->monopole) {
        const double ms = p->monopole_width;
        double sum = 0.0;
        for (int i = 0; i < n; ++i) {
            const double t = (i - n / 2) * pl->dt - p->center_shift * pl->dt;
            const double ph = std::exp(-t * t / (2.0 * ms * ms)) / (std::sqrt(2.0 * M_PI) * ms);
            mono_phi[i] = (float)ph;
            sum += ph;
        }
        pl->mono_inv = (float)(1.0 / ((double)V * sum));
        pl->mono_amp = (float)(M_PI / (std::sqrt(2.0 * M_PI) * ms));
        pl->mono_rho_px = (float)(d * d / (4.0 * ms * ms));
    }

    // ---- one device block ----
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_taper = off; off = up(off + n * sizeof(float));
    const size_t o_kc = off;    off = up(off + (M / 2) * sizeof(float2));
    const size_t o_twM = off;   off = up(off + M * sizeof(float2));
    const size_t o_twG = off;   off = up(off + G * sizeof(float2));
    const size_t o_c = off;     off = up(off + V * sizeof(double));
    const size_t o_s = off;     off = up(off + V * sizeof(double));
    const size_t o_w = off;     off = up(off + V * sizeof(float));
    const size_t o_ang = off;   off = up(off + V * sizeof(double2));
    const size_t o_gap = off;   off = up(off + V * sizeof(float));
    const size_t o_prow = off;  off = up(off + V * sizeof(float));
    const size_t o_mphi = off;  off = up(off + n * sizeof(float));
    const size_t o_ramp = off;  off = up(off + n * sizeof(double));
    const size_t o_tap64 = off; off = up(off + n * sizeof(double));
    const size_t o_kc64 = off;  off = up(off + (M / 2) * sizeof(double2));
    const size_t total = off;
    std::vector<unsigned char> host(total, 0);
    std::memcpy(host.data() + o_taper, taper.data(), n * sizeof(float));
    std::memcpy(host.data() + o_kc, kc.data(), (M / 2) * sizeof(float2));
    std::memcpy(host.data() + o_twM, twM.data(), M * sizeof(float2));
    std::memcpy(host.data() + o_twG, twG.data(), G * sizeof(float2));
    std::memcpy(host.data() + o_c, bf_c.data(), V * sizeof(double));
    std::memcpy(host.data() + o_s, bf_s.data(), V * sizeof(double));
    std::memcpy(host.data() + o_w, bf_w.data(), V * sizeof(float));
    std::memcpy(host.data() + o_ang, ang.data(), V * sizeof(double2));
    std::memcpy(host.data() + o_gap, inv_gap.data(), V * sizeof(float));
    std::memcpy(host.data() + o_prow, proj_row.data(), V * sizeof(float));
    std::memcpy(host.data() + o_mphi, mono_phi.data(), n * sizeof(float));
    // band-limited ramp of the brute-force comparison (Kak and Slaney): h[0] =
    // 1/(4 dt^2), h[d odd] = -1/(pi^2 d^2 dt^2), h[d even] = 0, times dt
    std::vector<double> ramp_h(n, 0.0);
    ramp_h[0] = 1.0 / (4.0 * pl->dt);
    for (int d = 1; d < n; d += 2) ramp_h[d] = -1.0 / (M_PI * M_PI * (double)d * (double)d * pl->dt);
    std::memcpy(host.data() + o_ramp, ramp_h.data(), n * sizeof(double));
    std::memcpy(host.data() + o_tap64, taper64.data(), n * sizeof(double));
    std::memcpy(host.data() + o_kc64, kc64.data(), (M / 2) * sizeof(double2));

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= p->device) {
        delete pl;
        if (e == hipSuccess) e = hipErrorInvalidDevice;
        return device_fail(e);
    }
    DeviceGuard guard(p->device);
    if (guard.err != hipSuccess) {
        delete pl;
        return device_fail(guard.err);
    }
    e = hipMalloc(&pl->dev_block, total);
    if (e != hipSuccess) {
        g_last_error = hipGetErrorString(e);
        delete pl;
        return BST_E_NOMEM;
    }
    e = hipMemcpy(pl->dev_block, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(pl->dev_block);
        delete pl;
        return device_fail(e);
    }
    std::vector<int2> tent_cols;
    if (pl->tent) {
        pl->tent_w = bst::tent_columns(G, V, tent_cols);
        pl->tent_rows = bst::tent_rows(V, M, pl->rscale);
        std::vector<int4> chunks;
        std::vector<int> coff;
        bst::tent_chunks(V, tent_cols, chunks, coff);
        pl->tent_chunks = chunks.size();
        const size_t o_chunk = up(tent_cols.size() * sizeof(int2));
        const size_t o_coff = up(o_chunk + std::max<size_t>(chunks.size(), 1) * sizeof(int4));
        const size_t t_total = o_coff + coff.size() * sizeof(int);
        e = hipMalloc(&pl->tent_block, t_total);
        if (e != hipSuccess) {
            g_last_error = hipGetErrorString(e);
            (void)hipFree(pl->dev_block);
            delete pl;
            return BST_E_NOMEM;
        }
        unsigned char* tb = static_cast<unsigned char*>(pl->tent_block);
        e = hipMemcpy(tb, tent_cols.data(), tent_cols.size() * sizeof(int2), hipMemcpyHostToDevice);
        if (e == hipSuccess && !chunks.empty())
            e = hipMemcpy(tb + o_chunk, chunks.data(), chunks.size() * sizeof(int4), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(tb + o_coff, coff.data(), coff.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(pl->tent_block);
            (void)hipFree(pl->dev_block);
            delete pl;
            return device_fail(e);
        }
        pl->tent_cols = reinterpret_cast<int2*>(tb);
        pl->tent_chunk = reinterpret_cast<int4*>(tb + o_chunk);
        pl->tent_coff = reinterpret_cast<int*>(tb + o_coff);
    }
    if (pl->adjoint) {
        std::vector<int> off;
        std::vector<uint2> ent;
        bst::build_adjoint_tables(V, M, G, pl->rscale, theta, pl->uniform, pl->taps,
                                  pl->tent ? &tent_cols : nullptr, off, ent);
        pl->n_entries = ent.size();
        const size_t o_ent = up(off.size() * sizeof(int));
        const size_t adj_total = o_ent + std::max<size_t>(ent.size(), 1) * sizeof(uint2);
        e = hipMalloc(&pl->adj_block, adj_total);
        if (e != hipSuccess) {
            g_last_error = hipGetErrorString(e);
            if (pl->tent_block) (void)hipFree(pl->tent_block);
            (void)hipFree(pl->dev_block);
            delete pl;
            return BST_E_NOMEM;
        }
        e = hipMemcpy(pl->adj_block, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e == hipSuccess && !ent.empty())
            e = hipMemcpy(static_cast<unsigned char*>(pl->adj_block) + o_ent, ent.data(),
                          ent.size() * sizeof(uint2), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(pl->adj_block);
            if (pl->tent_block) (void)hipFree(pl->tent_block);
            (void)hipFree(pl->dev_block);
            delete pl;
            return device_fail(e);
        }
        pl->csr_off = static_cast<int*>(pl->adj_block);
        pl->csr_ent = reinterpret_cast<uint2*>(static_cast<unsigned char*>(pl->adj_block) + o_ent);
    }
    unsigned char* base = static_cast<unsigned char*>(pl->dev_block);
    pl->taper = reinterpret_cast<float*>(base + o_taper);
    pl->kc = reinterpret_cast<float2*>(base + o_kc);
    pl->tw_M = reinterpret_cast<float2*>(base + o_twM);
    pl->tw_G = reinterpret_cast<float2*>(base + o_twG);
    pl->bf_c = reinterpret_cast<double*>(base + o_c);
    pl->bf_s = reinterpret_cast<double*>(base + o_s);
    pl->bf_w = reinterpret_cast<float*>(base + o_w);
    pl->ang = reinterpret_cast<double2*>(base + o_ang);
    pl->inv_gap = reinterpret_cast<float*>(base + o_gap);
    pl->proj_row = reinterpret_cast<float*>(base + o_prow);
    pl->mono_phi = reinterpret_cast<float*>(base + o_mphi);
    pl->ramp_h = reinterpret_cast<double*>(base + o_ramp);
    pl->taper64 = reinterpret_cast<double*>(base + o_tap64);
    pl->kc64 = reinterpret_cast<double2*>(base + o_kc64);
    *out = pl;
    return BST_OK;
}

bst_status bst_workspace_size(bst_plan_t plan, int32_t batch, size_t* bytes) {
    if (!plan || !bytes) return BST_E_NULL;
    if (batch < 0 || batch > plan->prm.max_batch) return BST_E_BATCH;
    *bytes = bst::workspace_bytes(plan->n, plan->V, plan->N, plan->M, plan->G, batch, plan->adjoint,
                                  plan->prm.interp, plan->monopole, tent_sizes(plan), plan->f64);
    return BST_OK;
}

}  // extern "C"

namespace {

bst_status check_call(bst_plan_t plan, const void* in, size_t in_bytes, const void* out, size_t out_bytes,
                      int32_t batch, const void* ws, size_t ws_bytes, bool need_ws, size_t* need) {
    if (!plan) return BST_E_NULL;
    if (batch < 0 || batch > plan->prm.max_batch) return BST_E_BATCH;
    if (batch == 0) return BST_OK;
    if (!in || !out) return BST_E_NULL;
    if (need_ws) {
        *need = bst::workspace_layout(plan->n, plan->V, plan->N, plan->M, plan->G, batch, plan->prm.interp,
                                      plan->monopole, tent_sizes(plan))
                    .total;
        if (!ws) return BST_E_NULL;
        if (ws_bytes < *need) return BST_E_WORKSPACE;
    }
    const Range ri{(uintptr_t)in, (uintptr_t)in + in_bytes};
    const Range ro{(uintptr_t)out, (uintptr_t)out + out_bytes};
    if (overlap(ri, ro)) return BST_E_ALIAS;
    if (need_ws) {
        const Range rw{(uintptr_t)ws, (uintptr_t)ws + *need};
        if (overlap(rw, ri) || overlap(rw, ro)) return BST_E_ALIAS;
    }
    return BST_OK;
}

bst_status run_backproject(bst_plan_t plan, const float* sino, float* img, int32_t batch, void* ws,
                           size_t ws_bytes, void* stream, void* const* ev, bool spectrum_only,
                           void* spec_out, float* dc_out, const float* flat = nullptr,
                           const float* dark = nullptr, const float* const* sino_list = nullptr,
                           float* const* img_list = nullptr) {
    if (!plan) return BST_E_NULL;
    if (plan->f64) return BST_E_UNSUPPORTED;  // bst_backproject_f64
    const size_t in_bytes = (size_t)batch * plan->V * plan->n * sizeof(float);
    const size_t out_bytes = (size_t)batch * plan->N * plan->N * sizeof(float);
    size_t need = 0;
    bst_status st;
    if (spectrum_only) {
        if (batch > 0 && (!spec_out || !dc_out)) return BST_E_NULL;
        st = check_call(plan, sino, in_bytes, spec_out,
                        (size_t)batch * plan->V * (plan->M / 2) * sizeof(float2), batch, ws, ws_bytes, true,
                        &need);
    } else {
        st = check_call(plan, sino, in_bytes, img, out_bytes, batch, ws, ws_bytes, true, &need);
    }
    if (st != BST_OK || batch == 0) return st;

    DeviceGuard guard(plan->device);
    if (guard.err != hipSuccess) return device_fail(guard.err);
    bst::TraceRange trace(spectrum_only ? "bst_debug_spectrum" : "bst_backproject");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bst::WsLayout L = bst::workspace_layout(plan->n, plan->V, plan->N, plan->M, plan->G, batch,
                                                  plan->prm.interp, plan->monopole, tent_sizes(plan));
    unsigned char* w = static_cast<unsigned char*>(ws);
    float2* polar = reinterpret_cast<float2*>(w + L.polar_off);
    float* dc = reinterpret_cast<float*>(w + L.dc_off);
    float2* grid = reinterpret_cast<float2*>(w + L.grid_off);
    float* mass = plan->monopole ? reinterpret_cast<float*>(w + L.mass_off) : nullptr;
    hipError_t e;

    if (ev && ev[0]) {
        e = hipEventRecord(static_cast<hipEvent_t>(ev[0]), s);
        if (e != hipSuccess) return device_fail(e);
    }
    if (plan->monopole) {
        bst::TraceRange tr("bst monopole mass");
        const bst::MassArgs ma{sino, sino_list, flat, dark, mass, plan->n, plan->V};
        e = bst::launch_mass(*plan, ma, batch, s);
        if (e != hipSuccess) return device_fail(e);
    }
    bst::SpecArgs sa{sino,   sino_list, flat,    dark,       polar,          dc,
                     plan->taper, plan->kc, plan->tw_M, plan->n, plan->V, plan->S,
                     plan->lead,  plan->S - plan->lead - plan->M / 2, (float)plan->dt,
                     mass, plan->mono_phi, plan->mono_inv};
    {
        bst::TraceRange tr("bst P1-P4 spectrum");
        e = bst::launch_spectrum(*plan, sa, batch, s);
    }
    if (e != hipSuccess) return device_fail(e);
    if (ev && ev[1]) {
        e = hipEventRecord(static_cast<hipEvent_t>(ev[1]), s);
        if (e != hipSuccess) return device_fail(e);
    }
    if (spectrum_only) {
        e = bst::launch_polar_extract(*plan, polar, static_cast<float2*>(spec_out), batch, s);
        if (e != hipSuccess) return device_fail(e);
        e = hipMemcpyAsync(dc_out, dc, (size_t)batch * plan->V * sizeof(float), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return device_fail(e);
        return BST_OK;
    }
    bst::GatherArgs ga{};
    ga.polar = polar;
    ga.dc = dc;
    ga.grid = grid;
    ga.tw = plan->tw_G;
    ga.V = plan->V;
    ga.S = plan->S;
    ga.GT = plan->GT;
    ga.N = plan->N;
    ga.Mh = plan->M / 2;
    ga.zero_slot = plan->M / 2 + plan->lead;
    ga.batch = batch;
    ga.slices_per_block = plan->gather_slices;
    ga.rscale = plan->rscale;
    ga.vpi_f = (float)plan->vpi;
    ga.ang = plan->ang;
    ga.inv_gap = plan->inv_gap;
    ga.uniform = plan->uniform ? 1 : 0;
    ga.dc_scale = plan->dc_scale;
    if (plan->tent) {
        float2* patch = reinterpret_cast<float2*>(w + L.tent_off);
        float2* trans = reinterpret_cast<float2*>(w + L.tent_trans_off);
        float2* part = reinterpret_cast<float2*>(w + L.tent_part_off);
        float* wsum = reinterpret_cast<float*>(w + L.tent_wsum_off);
        const bst::TentArgs ta{polar, trans, patch, part, wsum, plan->tent_cols, plan->tent_chunk, plan->tent_coff,
                               (int)plan->tent_w, (int)plan->tent_chunks, plan->V, plan->S, plan->lead,
                               plan->tent_rows, plan->G / 2, plan->rscale};
        bst::TraceRange tr("bst P5 tent pre-gather");
        e = bst::launch_tent(*plan, ta, batch, s);
        if (e != hipSuccess) return device_fail(e);
        ga.tent_cols = plan->tent_cols;
        ga.patch = patch;
        ga.tent_w = (int)plan->tent_w;
    }
    {
        bst::TraceRange tr("bst P5-P6 gather + column IFFT");
        e = bst::launch_gather_colifft(*plan, ga, s);
    }
    if (e != hipSuccess) return device_fail(e);
    if (ev && ev[2]) {
        e = hipEventRecord(static_cast<hipEvent_t>(ev[2]), s);
        if (e != hipSuccess) return device_fail(e);
    }
    bst::RowArgs ra{grid, img, img_list, plan->tw_G, plan->N, plan->GT, plan->out_scale, 0,
                    mass, plan->mono_inv, plan->mono_amp, plan->mono_rho_px};
    {
        bst::TraceRange tr("bst P6-P8 row C2R + crop");
        e = bst::launch_row_c2r(*plan, ra, batch, s);
    }
    if (e != hipSuccess) return device_fail(e);
    if (ev && ev[3]) {
        e = hipEventRecord(static_cast<hipEvent_t>(ev[3]), s);
        if (e != hipSuccess) return device_fail(e);
    }
    return BST_OK;
}

}  // namespace

namespace bst {
size_t backproject_workspace_need(bst_plan_t plan, int32_t batch) {
    if (!plan || batch <= 0) return 0;
    return workspace_layout(plan->n, plan->V, plan->N, plan->M, plan->G, batch, plan->prm.interp, plan->monopole,
                            tent_sizes(plan))
        .total;
}

bst_status backproject_in(bst_plan_t plan, const float* sino, float* img, int32_t batch, void* ws,
                          size_t ws_bytes, void* stream) {
    return run_backproject(plan, sino, img, batch, ws, ws_bytes, stream, nullptr, false, nullptr, nullptr);
}

void set_last_error_text(const char* text) { g_last_error = text; }
}  // namespace bst

extern "C" {

bst_status bst_backproject(bst_plan_t plan, const float* sino, float* img, int32_t batch, void* ws,
                           size_t ws_bytes, void* stream) {
    return run_backproject(plan, sino, img, batch, ws, ws_bytes, stream, nullptr, false, nullptr, nullptr);
}

bst_status bst_backproject_counts(bst_plan_t plan, const float* counts, const float* flat, const float* dark,
                                  float* img, int32_t batch, void* ws, size_t ws_bytes, void* stream) {
    if (!plan) return BST_E_NULL;
    if (batch > 0 && (!flat || !dark)) return BST_E_NULL;
    if (batch > 0 && batch <= plan->prm.max_batch) {
        const size_t fb = (size_t)batch * plan->n * sizeof(float);
        const Range rf{(uintptr_t)flat, (uintptr_t)flat + fb}, rd{(uintptr_t)dark, (uintptr_t)dark + fb};
        const Range ro{(uintptr_t)img, (uintptr_t)img + (size_t)batch * plan->N * plan->N * sizeof(float)};
        if (overlap(rf, ro) || overlap(rd, ro)) return BST_E_ALIAS;
    }
    return run_backproject(plan, counts, img, batch, ws, ws_bytes, stream, nullptr, false, nullptr, nullptr, flat,
                           dark);
}

bst_status bst_backproject_timed(bst_plan_t plan, const float* sino, float* img, int32_t batch, void* ws,
                                 size_t ws_bytes, void* stream, void* const* events4) {
    if (!events4) return BST_E_NULL;
    for (int i = 0; i < 4; ++i)
        if (!events4[i]) return BST_E_NULL;
    return run_backproject(plan, sino, img, batch, ws, ws_bytes, stream, events4, false, nullptr, nullptr);
}

bst_status bst_debug_spectrum(bst_plan_t plan, const float* sino, void* spec, float* dc, int32_t batch,
                              void* ws, size_t ws_bytes, void* stream) {
    return run_backproject(plan, sino, nullptr, batch, ws, ws_bytes, stream, nullptr, true, spec, dc);
}

bst_status bst_backproject_bruteforce(bst_plan_t plan, const float* sino, float* img, int32_t batch,
                                      void* stream) {
    if (!plan) return BST_E_NULL;
    const size_t in_bytes = (size_t)batch * plan->V * plan->n * sizeof(float);
    const size_t out_bytes = (size_t)batch * plan->N * plan->N * sizeof(float);
    size_t need = 0;
    const bst_status st = check_call(plan, sino, in_bytes, img, out_bytes, batch, nullptr, 0, false, &need);
    if (st != BST_OK || batch == 0) return st;
    DeviceGuard guard(plan->device);
    if (guard.err != hipSuccess) return device_fail(guard.err);
    bst::BfArgs a{sino, img, plan->bf_c, plan->bf_s, plan->bf_w, plan->n, plan->V, plan->N};
    bst::TraceRange tr("bst_backproject_bruteforce");
    const hipError_t e = bst::launch_bruteforce(*plan, a, batch, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_fail(e);
    return BST_OK;
}

namespace {
// the FP64 path's call: checks, workspace carving, kernels (B or R)
bst_status run_f64(bst_plan_t plan, const double* in, double* out, int32_t batch, void* ws, size_t ws_bytes,
                   void* stream, bool project) {
    if (!plan) return BST_E_NULL;
    if (!plan->f64) return BST_E_UNSUPPORTED;
    if (batch < 0 || batch > plan->prm.max_batch) return BST_E_BATCH;
    if (batch == 0) return BST_OK;
    if (!in || !out || !ws) return BST_E_NULL;
    const bst::F64WsLayout L = bst::f64_workspace_layout(plan->V, plan->M, plan->G, batch);
    if (ws_bytes < L.total) return BST_E_WORKSPACE;
    const size_t sino_bytes = (size_t)batch * plan->V * plan->n * sizeof(double);
    const size_t img_bytes = (size_t)batch * plan->N * plan->N * sizeof(double);
    const Range ri{(uintptr_t)in, (uintptr_t)in + (project ? img_bytes : sino_bytes)};
    const Range ro{(uintptr_t)out, (uintptr_t)out + (project ? sino_bytes : img_bytes)};
    const Range rw{(uintptr_t)ws, (uintptr_t)ws + L.total};
    if (overlap(ri, ro) || overlap(rw, ri) || overlap(rw, ro)) return BST_E_ALIAS;
    DeviceGuard guard(plan->device);
    if (guard.err != hipSuccess) return device_fail(guard.err);
    unsigned char* w = static_cast<unsigned char*>(ws);
    bst::F64Args a{};
    a.polar = reinterpret_cast<double2*>(w + L.polar_off);
    a.dc = reinterpret_cast<double*>(w + L.dc_off);
    a.cart = reinterpret_cast<double2*>(w + L.cart_off);
    a.polar_t = reinterpret_cast<double2*>(w + L.polar_t_off);
    a.origin = reinterpret_cast<double*>(w + L.origin_off);
    a.taper = plan->taper64;
    a.kc = plan->kc64;
    a.n = plan->n;
    a.V = plan->V;
    a.N = plan->N;
    a.M = plan->M;
    a.G = plan->G;
    a.dt = plan->dt;
    a.dk2 = plan->dk * plan->dk;
    a.rscale = plan->rscale;
    a.dc_rule = plan->prm.filter == BST_FILTER_RAMP ? 1.0 : 4.0 * std::asinh(1.0) / plan->dk;
    const double d = 2.0 / plan->N;
    a.row_scale = d * d / (plan->dt * M_PI / plan->V);
    hipError_t e;
    if (project) {
        a.img_in = in;
        a.sino = out;
        bst::TraceRange tr("bst_project_f64");
        e = bst::launch_fp64_project(a, batch, static_cast<hipStream_t>(stream));
    } else {
        a.sino_in = in;
        a.img = out;
        bst::TraceRange tr("bst_backproject_f64");
        e = bst::launch_fp64_backproject(a, batch, static_cast<hipStream_t>(stream));
    }
    return e == hipSuccess ? BST_OK : device_fail(e);
}
}  // namespace

bst_status bst_backproject_f64(bst_plan_t plan, const double* sino, double* img, int32_t batch, void* ws,
                               size_t ws_bytes, void* stream) {
    return run_f64(plan, sino, img, batch, ws, ws_bytes, stream, false);
}

bst_status bst_project_f64(bst_plan_t plan, const double* img, double* sino, int32_t batch, void* ws,
                           size_t ws_bytes, void* stream) {
    return run_f64(plan, img, sino, batch, ws, ws_bytes, stream, true);
}

bst_status bst_ramp_filter(bst_plan_t plan, const float* sino, float* out, int32_t batch, void* stream) {
    if (!plan) return BST_E_NULL;
    const size_t bytes = (size_t)batch * plan->V * plan->n * sizeof(float);
    size_t need = 0;
    const bst_status st = check_call(plan, sino, bytes, out, bytes, batch, nullptr, 0, false, &need);
    if (st != BST_OK || batch == 0) return st;
    DeviceGuard guard(plan->device);
    if (guard.err != hipSuccess) return device_fail(guard.err);
    const bst::RampArgs a{sino, out, plan->ramp_h, plan->n, plan->V};
    bst::TraceRange tr("bst_ramp_filter");
    const hipError_t e = bst::launch_ramp_filter(*plan, a, batch, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? BST_OK : device_fail(e);
}

bst_status bst_project(bst_plan_t plan, const float* img, float* sino, int32_t batch, void* ws,
                       size_t ws_bytes, void* stream) {
    if (!plan) return BST_E_NULL;
    const size_t in_bytes = (size_t)batch * plan->N * plan->N * sizeof(float);
    const size_t out_bytes = (size_t)batch * plan->V * plan->n * sizeof(float);
    if (batch < 0 || batch > plan->prm.max_batch) return BST_E_BATCH;
    if (batch == 0) return BST_OK;
    if (!img || !sino || !ws) return BST_E_NULL;
    if (!plan->adjoint || plan->f64) return BST_E_UNSUPPORTED;
    const bst::ProjWsLayout L = bst::project_workspace_layout(plan->V, plan->N, plan->M, plan->G, batch);
    if (ws_bytes < L.total) return BST_E_WORKSPACE;
    const Range ri{(uintptr_t)img, (uintptr_t)img + in_bytes};
    const Range ro{(uintptr_t)sino, (uintptr_t)sino + out_bytes};
    const Range rw{(uintptr_t)ws, (uintptr_t)ws + L.total};
    if (overlap(ri, ro) || overlap(rw, ri) || overlap(rw, ro)) return BST_E_ALIAS;

    DeviceGuard guard(plan->device);
    if (guard.err != hipSuccess) return device_fail(guard.err);
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char* w = static_cast<unsigned char*>(ws);
    float2* grid = reinterpret_cast<float2*>(w + L.grid_off);
    float2* cart8 = reinterpret_cast<float2*>(w + L.cart8_off);
    float2* polar = reinterpret_cast<float2*>(w + L.polar_off);
    const int cart_stride = (plan->G / 2) * plan->G;

    bst::ProjRowArgs ra{img, grid, plan->tw_G, plan->N, plan->out_scale};
    bst::TraceRange tr("bst_project");
    hipError_t e = bst::launch_proj_rows(*plan, ra, batch, s);
    if (e != hipSuccess) return device_fail(e);
    const int groups = (batch + bst::kProjInterleave - 1) / bst::kProjInterleave;
    bst::ProjColArgs ca{grid, cart8, plan->tw_G, plan->N, batch, groups * (plan->G / 2)};
    e = bst::launch_proj_cols(*plan, ca, batch, s);
    if (e != hipSuccess) return device_fail(e);
    bst::ProjGatherArgs ga{cart8, polar, plan->csr_off, plan->csr_ent, plan->V * (plan->M / 2), cart_stride,
                           batch, plan->M / 2};
    e = bst::launch_proj_gather(*plan, ga, s);
    if (e != hipSuccess) return device_fail(e);
    bst::ProjPolarArgs pa{polar, cart8, sino, plan->taper, plan->kc, plan->tw_M, plan->n, plan->V,
                          cart_stride, (float)(plan->dt * plan->dc_scale), plan->proj_row};
    e = bst::launch_proj_polar(*plan, pa, batch, s);
    if (e != hipSuccess) return device_fail(e);
    return BST_OK;
}

bst_status bst_destroy(bst_plan_t plan) {
    if (!plan) return BST_OK;
    bst_status st = BST_OK;
    if (plan->dev_block || plan->adj_block || plan->tent_block) {
        DeviceGuard guard(plan->device);
        for (void* blk : {plan->dev_block, plan->adj_block, plan->tent_block}) {
            if (!blk) continue;
            const hipError_t e = hipFree(blk);
            if (e != hipSuccess) st = device_fail(e);
        }
    }
    delete plan;
    return st;
}

const char* bst_status_string(int32_t status) {
    // switch on the integer: a value outside the enumerators is not a valid bst_status in C++
    switch (status) {
        case BST_OK: return "ok";
        case BST_E_NULL: return "null pointer argument";
        case BST_E_SHAPE: return "unsupported or inconsistent sizes";
        case BST_E_ANGLES: return "angles must be finite, strictly increasing and in [0, pi)";
        case BST_E_PARAM: return "invalid filter, taper, padding or device value";
        case BST_E_WORKSPACE: return "workspace smaller than bst_workspace_size";
        case BST_E_NOMEM: return "device allocation failed";
        case BST_E_DEVICE: return "HIP runtime error";
        case BST_E_UNSUPPORTED: return "not supported by the library as compiled";
        case BST_E_BATCH: return "batch out of range [0, max_batch]";
        case BST_E_ALIAS: return "input, output and workspace must not overlap";
    }
    return "unknown status";
}

const char* bst_last_error_string(void) { return g_last_error.c_str(); }

bst_status bst_debug_check(int32_t device, uint32_t* flags) {
    if (!flags) return BST_E_NULL;
    *flags = 0;
#ifdef BST_CHECKED
    DeviceGuard guard(device);
    if (guard.err != hipSuccess) return device_fail(guard.err);
    const unsigned parts[4] = {bst::check_flags_spectrum(), bst::check_flags_gather(), bst::check_flags_row(),
                               bst::check_flags_project()};
    for (int i = 0; i < 4; ++i) {
        if (parts[i] == ~0u) return BST_E_DEVICE;
        *flags |= (parts[i] & 0xFFu) << (8 * i);
    }
    return BST_OK;
#else
    (void)device;
    return BST_E_UNSUPPORTED;
#endif
}

bst_status bst_event_create(void** ev) {
    if (!ev) return BST_E_NULL;
    hipEvent_t e = nullptr;
    const hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return device_fail(r);
    *ev = e;
    return BST_OK;
}

bst_status bst_event_destroy(void* ev) {
    if (!ev) return BST_OK;
    const hipError_t r = hipEventDestroy(static_cast<hipEvent_t>(ev));
    return r == hipSuccess ? BST_OK : device_fail(r);
}

bst_status bst_event_elapsed_ms(void* start, void* stop, float* ms) {
    if (!start || !stop || !ms) return BST_E_NULL;
    const hipError_t r = hipEventElapsedTime(ms, static_cast<hipEvent_t>(start), static_cast<hipEvent_t>(stop));
    return r == hipSuccess ? BST_OK : device_fail(r);
}

bst_status bst_stream_synchronize(void* stream) {
    const hipError_t r = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    return r == hipSuccess ? BST_OK : device_fail(r);
}

}  // extern "C"
