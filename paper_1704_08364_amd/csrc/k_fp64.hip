// k_fp64.hip -- the FP64 gradient-check path: the BST backprojection B
// (Section 2, steps P1-P8) and its exact adjoint R in double precision, for
// plans built with dtype BST_F64 (n <= 512, uniform angles, linear radial and
// angular interpolation). These kernels favour plainness over speed: they
// exist so that gradients of least-squares objectives can be checked against
// finite differences with FP64 round-off, and B and R against the FP64 oracle
// to ~1e-12.
//
// Every transform is a radix-2 FFT of one line held in LDS by one block
// (bit-reversed load, log2 L in-place butterfly stages, twiddles from FP64
// sincospi). Data layouts (complex = double2):
//   polar   [B][V][M/2 + 2]   Yh = K A phase dt Y, two zero slots at the end
//   dc      [B][V]            dt Y_j[0]
//   cart    [B][G][G/2 + 1]   row b (FFT order), column a (half plane)
//   polar_t [B][V][M/2 + 1]   the adjoint's polar accumulator
#include "bst_internal.h"

namespace bst {

constexpr int kF64Threads = 256;

// y <- forward (sign = -1) or inverse (sign = +1, unnormalised) DFT of the L
// values in x (LDS), L a power of two; all threads of the block take part.
__device__ void fft64_lds(double2* x, int L, int sign) {
    // bit-reversal permutation in place
    const int bits = __ffs(L) - 1;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        const int r = (int)(__brev((unsigned)i) >> (32 - bits));
        if (r > i) {
            const double2 t = x[i];
            x[i] = x[r];
            x[r] = t;
        }
    }
    __syncthreads();
    for (int len = 2; len <= L; len <<= 1) {
        const int half = len >> 1;
        for (int t = threadIdx.x; t < L / 2; t += blockDim.x) {
            const int grp = t / half, k = t - grp * half;
            const int i0 = grp * len + k, i1 = i0 + half;
            double sn, cs;
            sincospi((double)sign * 2.0 * (double)k / (double)len, &sn, &cs);
            const double2 b = x[i1];
            const double2 w = make_double2(b.x * cs - b.y * sn, b.x * sn + b.y * cs);
            const double2 a = x[i0];
            x[i0] = make_double2(a.x + w.x, a.y + w.y);
            x[i1] = make_double2(a.x - w.x, a.y - w.y);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ double2 cmul64(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 conj64(double2 a, bool c) { return c ? make_double2(a.x, -a.y) : a; }

// ---- B ----------------------------------------------------------------------

// P1-P4 for one projection: taper, centred zero padding, FFT, radial weight.
__global__ void __launch_bounds__(kF64Threads) k64_spectrum(F64Args a) {
    extern __shared__ double2 z[];
    const int j = blockIdx.x, s = blockIdx.y;
    const int M = a.M, n = a.n;
    const double* y = a.sino_in + ((size_t)s * a.V + j) * n;
    for (int k = threadIdx.x; k < M; k += blockDim.x) z[k] = make_double2(0.0, 0.0);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) z[(i - n / 2 + M) % M].x = a.taper[i] * y[i];
    __syncthreads();
    fft64_lds(z, M, -1);
    double2* row = a.polar + ((size_t)s * a.V + j) * (M / 2 + 2);
    for (int m = threadIdx.x; m < M / 2 + 2; m += blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        if (m < M / 2) v = cmul64(make_double2(a.dt * z[m].x, a.dt * z[m].y), a.kc[m]);
        row[m] = v;
    }
    if (threadIdx.x == 0) a.dc[(size_t)s * a.V + j] = a.dt * z[0].x;
}

// Stencil of Cartesian point (a, b) (b signed): the two angle rows, radial tap
// and weights of the bilinear gather in (radius, angle index), FP64.
struct Stencil64 {
    int j0, j1, m0;
    double f, g;
    bool c0, c1;  // conjugation of the j0 and j1 samples
};
__device__ Stencil64 stencil64(int a, int b, const F64Args& p) {
    Stencil64 st;
    const double r = sqrt((double)a * a + (double)b * b) * p.rscale;
    const double phi = atan2((double)b, (double)a);
    const bool lower = phi < 0.0;
    const double theta = lower ? phi + M_PI : phi;
    const double q = theta * ((double)p.V / M_PI);
    const double j0 = floor(q);
    st.f = q - j0;
    st.j0 = (int)j0;
    if (st.j0 >= p.V) {  // rounding guard: theta == pi
        st.j0 = p.V - 1;
        st.f = 1.0;
    }
    const bool wrap = st.j0 + 1 >= p.V;
    st.j1 = wrap ? 0 : st.j0 + 1;
    st.c0 = lower;
    st.c1 = lower != wrap;
    const double mf = floor(r);
    st.m0 = (int)mf;
    st.g = r - mf;
    return st;
}

// P5: the Cartesian half plane, one thread per point (row b, column a).
__global__ void __launch_bounds__(kF64Threads) k64_gather(F64Args a) {
    const int G = a.G, W = G / 2 + 1;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (idx >= (size_t)G * W) return;
    const int bi = (int)(idx / W), ai = (int)(idx % W);
    const int bs = bi < G / 2 ? bi : bi - G;
    double2 v = make_double2(0.0, 0.0);
    if (ai == 0 && bs == 0) {
        // origin rule: dc_rule * mean_j dt Y_j[0]
        double acc = 0.0;
        for (int j = 0; j < a.V; ++j) acc += a.dc[(size_t)s * a.V + j];
        v.x = a.dc_rule * acc / (double)a.V;
    } else if (ai < G / 2) {
        const Stencil64 st = stencil64(ai, bs, a);
        const double2* P = a.polar + (size_t)s * a.V * (a.M / 2 + 2);
        auto S = [&](int j, int m, bool c) {
            return m < a.M / 2 ? conj64(P[(size_t)j * (a.M / 2 + 2) + m], c) : make_double2(0.0, 0.0);
        };
        const double2 s00 = S(st.j0, st.m0, st.c0), s01 = S(st.j0, st.m0 + 1, st.c0);
        const double2 s10 = S(st.j1, st.m0, st.c1), s11 = S(st.j1, st.m0 + 1, st.c1);
        const double w00 = (1 - st.f) * (1 - st.g), w01 = (1 - st.f) * st.g;
        const double w10 = st.f * (1 - st.g), w11 = st.f * st.g;
        v.x = w00 * s00.x + w01 * s01.x + w10 * s10.x + w11 * s11.x;
        v.y = w00 * s00.y + w01 * s01.y + w10 * s10.y + w11 * s11.y;
    }
    a.cart[(size_t)s * G * W + idx] = v;
}

// P6 (columns): inverse DFT along b of every column a of the half plane, in place.
__global__ void __launch_bounds__(kF64Threads) k64_columns(F64Args a, int sign) {
    extern __shared__ double2 x[];
    const int G = a.G, W = G / 2 + 1;
    const int col = blockIdx.x, s = blockIdx.y;
    double2* C = a.cart + (size_t)s * G * W + col;
    for (int b = threadIdx.x; b < G; b += blockDim.x) x[b] = C[(size_t)b * W];
    __syncthreads();
    fft64_lds(x, G, sign);
    for (int b = threadIdx.x; b < G; b += blockDim.x) C[(size_t)b * W] = x[b];
}

// P6 (rows) + P7/P8: C2R along a of the N rows that survive the crop, times
// dk^2, cropped and shifted: img[p][q] = full[(p - N/2) mod G][(q - N/2) mod G].
__global__ void __launch_bounds__(kF64Threads) k64_rows_c2r(F64Args a) {
    extern __shared__ double2 x[];
    const int G = a.G, W = G / 2 + 1, N = a.N;
    const int p = blockIdx.x, s = blockIdx.y;
    const int y = (p - N / 2 + G) % G;
    const double2* R = a.cart + ((size_t)s * G + y) * W;
    // Hermitian extension; the imaginary parts of columns 0 and G/2 are dropped
    for (int k = threadIdx.x; k < G; k += blockDim.x) {
        double2 v;
        if (k == 0 || k == G / 2) v = make_double2(R[k].x, 0.0);
        else if (k < G / 2) v = R[k];
        else v = conj64(R[G - k], true);
        x[k] = v;
    }
    __syncthreads();
    fft64_lds(x, G, +1);
    double* out = a.img + ((size_t)s * N + p) * N;
    for (int q = threadIdx.x; q < N; q += blockDim.x) out[q] = a.dk2 * x[(q - N / 2 + G) % G].x;
}

// ---- R: the transposes, in reverse order ------------------------------------

// transpose of P8/P7 and the row C2R: image row p zero-embedded at full-grid
// row (p - N/2) mod G, column (q - N/2) mod G, forward DFT along a, columns
// 0..G/2 kept and scaled by dk^2 c_a (c_a = 1 for a in {0, G/2}, else 2).
// Full-grid rows outside the crop are zero.
__global__ void __launch_bounds__(kF64Threads) k64_rows_r2c(F64Args a) {
    extern __shared__ double2 x[];
    const int G = a.G, W = G / 2 + 1, N = a.N;
    const int yrow = blockIdx.x, s = blockIdx.y;
    const int p = (yrow + N / 2) % G;  // image row stored at full-grid row yrow, if p < N
    double2* R = a.cart + ((size_t)s * G + yrow) * W;
    if (p >= N) {
        for (int k = threadIdx.x; k < W; k += blockDim.x) R[k] = make_double2(0.0, 0.0);
        return;
    }
    for (int k = threadIdx.x; k < G; k += blockDim.x) x[k] = make_double2(0.0, 0.0);
    __syncthreads();
    const double* in = a.img_in + ((size_t)s * N + p) * N;
    for (int q = threadIdx.x; q < N; q += blockDim.x) x[(q - N / 2 + G) % G].x = in[q];
    __syncthreads();
    fft64_lds(x, G, -1);
    for (int k = threadIdx.x; k < W; k += blockDim.x) {
        const double c = (k == 0 || k == G / 2) ? 1.0 : 2.0;
        R[k] = make_double2(a.dk2 * c * x[k].x, a.dk2 * c * x[k].y);
    }
}

// clears the adjoint's polar accumulator (a kernel, not a memset, so that
// callers may capture the projector in a graph)
__global__ void __launch_bounds__(kF64Threads) k64_zero(double2* p, size_t count) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = make_double2(0.0, 0.0);
}

// transpose of the bilinear gather: every Cartesian point adds its value,
// weighted and conjugated as it was read, to its four polar samples (FP64
// atomics); the origin's rule goes to the origin term.
__global__ void __launch_bounds__(kF64Threads) k64_scatter(F64Args a) {
    const int G = a.G, W = G / 2 + 1;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (idx >= (size_t)G * W) return;
    const int bi = (int)(idx / W), ai = (int)(idx % W);
    const int bs = bi < G / 2 ? bi : bi - G;
    const double2 v = a.cart[(size_t)s * G * W + idx];
    if (ai == 0 && bs == 0) {
        a.origin[s] = v.x;
        return;
    }
    if (ai >= G / 2) return;
    const Stencil64 st = stencil64(ai, bs, a);
    double2* P = a.polar_t + (size_t)s * a.V * (a.M / 2 + 1);
    auto add = [&](int j, int m, bool c, double w) {
        if (m >= a.M / 2 || w == 0.0) return;
        const double2 t = conj64(v, c);
        double* d = reinterpret_cast<double*>(P + (size_t)j * (a.M / 2 + 1) + m);
        atomicAdd(d, w * t.x);
        atomicAdd(d + 1, w * t.y);
    };
    add(st.j0, st.m0, st.c0, (1 - st.f) * (1 - st.g));
    add(st.j0, st.m0 + 1, st.c0, (1 - st.f) * st.g);
    add(st.j1, st.m0, st.c1, st.f * (1 - st.g));
    add(st.j1, st.m0 + 1, st.c1, st.f * st.g);
}

// transpose of P4..P1 for one projection: conj(weight), plus the origin rule's
// share on m = 0, the transpose of the real DFT (dt * Re of the unnormalised
// inverse DFT of samples 0..M/2), crop of the padding, taper, d^2/(dt w).
__global__ void __launch_bounds__(kF64Threads) k64_polar_to_sino(F64Args a) {
    extern __shared__ double2 x[];
    const int M = a.M, n = a.n;
    const int j = blockIdx.x, s = blockIdx.y;
    const double2* P = a.polar_t + ((size_t)s * a.V + j) * (M / 2 + 1);
    for (int m = threadIdx.x; m < M; m += blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        if (m <= M / 2) {
            const double2 w = m < M / 2 ? a.kc[m] : make_double2(0.0, 0.0);
            v = cmul64(P[m], make_double2(w.x, -w.y));
            if (m == 0) v.x += a.dc_rule / (double)a.V * a.origin[s];
        }
        x[m] = v;
    }
    __syncthreads();
    fft64_lds(x, M, +1);
    double* out = a.sino + ((size_t)s * a.V + j) * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        out[i] = a.dt * x[(i - n / 2 + M) % M].x * a.taper[i] * a.row_scale;
}

hipError_t launch_fp64_backproject(const F64Args& a, int batch, hipStream_t st) {
    const int G = a.G, W = G / 2 + 1;
    const size_t pts = (size_t)G * W;
    hipLaunchKernelGGL(k64_spectrum, dim3(a.V, batch), dim3(kF64Threads), a.M * sizeof(double2), st, a);
    hipLaunchKernelGGL(k64_gather, dim3((unsigned)((pts + kF64Threads - 1) / kF64Threads), batch),
                       dim3(kF64Threads), 0, st, a);
    hipLaunchKernelGGL(k64_columns, dim3(W, batch), dim3(kF64Threads), G * sizeof(double2), st, a, +1);
    hipLaunchKernelGGL(k64_rows_c2r, dim3(a.N, batch), dim3(kF64Threads), G * sizeof(double2), st, a);
    return hipGetLastError();
}

hipError_t launch_fp64_project(const F64Args& a, int batch, hipStream_t st) {
    const int G = a.G, W = G / 2 + 1;
    const size_t pts = (size_t)G * W;
    hipLaunchKernelGGL(k64_rows_r2c, dim3(G, batch), dim3(kF64Threads), G * sizeof(double2), st, a);
    hipLaunchKernelGGL(k64_columns, dim3(W, batch), dim3(kF64Threads), G * sizeof(double2), st, a, -1);
    const size_t acc = (size_t)batch * a.V * (a.M / 2 + 1);
    hipLaunchKernelGGL(k64_zero, dim3((unsigned)((acc + kF64Threads - 1) / kF64Threads)), dim3(kF64Threads), 0, st,
                       a.polar_t, acc);
    hipLaunchKernelGGL(k64_scatter, dim3((unsigned)((pts + kF64Threads - 1) / kF64Threads), batch),
                       dim3(kF64Threads), 0, st, a);
    hipLaunchKernelGGL(k64_polar_to_sino, dim3(a.V, batch), dim3(kF64Threads), a.M * sizeof(double2), st, a);
    return hipGetLastError();
}

}  // namespace bst
