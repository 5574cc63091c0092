// k_gather_colifft.hip -- step P5 (polar -> Cartesian interpolation in the
// frequency domain, Section 2) fused with the first half of P6 (the inverse
// DFT along k_y) and the row part of P7/P8 (shift and crop).
//
// A block owns one Cartesian column k_x = a*dk (a in [0, G/2)) -- or several
// for small G -- and all G rows k_y = b*dk, b in FFT order. Each thread keeps
// the interpolation coordinates of its 16 points in registers: they are
// computed once in FP64 (radius index r = |(a,b)| P_r/P_c, angle index
// q = theta V/pi), which keeps the fractional weights exact to FP32 rounding
// even where r and q are near 3000, and reused for every slice the block
// processes. Per slice the column is gathered straight into the registers
// the FFT starts from, inverse-transformed along b, and only the N rows that
// survive the crop are written, to a grid laid out [N/8][G/2][8] (complex) so
// each group of 8 output rows of one column is a 64-byte segment and the row
// kernel reads its 8-row tile contiguously.
//
// Gather rules (bilinear in (r, q)):
//   b >= 0: theta = atan2(b, a), sample as stored; b < 0: theta + pi, conjugate
//   (y(t, theta + pi) = y(-t, theta)); the angle neighbour past theta_{V-1}
//   is theta_0 with the conjugation flipped; radial samples m >= M/2 are zero.
//   Origin (0,0): dc_scale * sum_j dt*Y_j[0] (mean for FBP, kappa/dk * mean
//   for plain B).
#include "bst_internal.h"
#include "fft_lds.h"

namespace bst {

constexpr int kZero = -1;
constexpr int kDc = -2;
constexpr int kConj = 1 << 30;
constexpr int kOffMask = kConj - 1;

template <int LOGG>
struct GatherCfg {
    static constexpr int G = 1 << LOGG;
    static constexpr int T = G / 16;
    static constexpr int F = T >= 256 ? 1 : 256 / T;   // columns per block
    static constexpr int WG = F * T;
};

template <int WG>
__device__ float block_sum(float x, float* red) {
    // deterministic: fixed-order wave reduction, then a fixed-order sum of wave totals
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    constexpr int NW = (WG + 63) / 64;
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = x;
    __syncthreads();
    float t = 0.f;
#pragma unroll
    for (int i = 0; i < NW; ++i) t += red[i];
    __syncthreads();
    return t;
}

template <int LOGG>
__global__ void __launch_bounds__(GatherCfg<LOGG>::WG) k_gather_colifft(GatherArgs a) {
    using C = GatherCfg<LOGG>;
    constexpr int G = C::G, T = C::T;
    __shared__ float2 lds[C::F * FftShape<LOGG>::LDS];
    __shared__ float red[(C::WG + 63) / 64];
    const int fid = threadIdx.x / T;
    const int j = threadIdx.x - fid * T;
    float2* my = lds + fid * FftShape<LOGG>::LDS;
    const int col = blockIdx.x * C::F + fid;
    const bool live = col < G / 2;

    int off0[16], off1[16];
    float fr[16], gr[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int b = j + e * T;
        const int bs = b < G / 2 ? b : b - G;
        off0[e] = kZero;
        off1[e] = 0;
        fr[e] = 0.f;
        gr[e] = 0.f;
        if (!live) continue;
        if (col == 0 && bs == 0) { off0[e] = kDc; continue; }
        const double r = sqrt((double)(col * col + bs * bs)) * a.rscale;
        if (r >= (double)a.Mh) continue;
        const double phi = atan2((double)bs, (double)col);
        const bool lower = phi < 0.0;
        const double th = lower ? phi + M_PI : phi;
        const double q = th * a.vpi;
        const double qf = floor(q);
        double f = q - qf;
        int j0 = (int)qf;
        if (j0 >= a.V) { j0 = a.V - 1; f = 1.0; }
        int j1 = j0 + 1;
        const bool wrap = (j1 == a.V);
        if (wrap) j1 = 0;
        const double mf = floor(r);
        const int m0 = (int)mf;
        off0[e] = (j0 * a.S + m0) | (lower ? kConj : 0);
        off1[e] = (j1 * a.S + m0) | ((lower != wrap) ? kConj : 0);
        fr[e] = (float)f;
        gr[e] = (float)(r - mf);
    }

    const int s_begin = blockIdx.y * a.slices_per_block;
    const int s_end = min(a.batch, s_begin + a.slices_per_block);
    const int half_n = a.N >> 1;
    for (int s = s_begin; s < s_end; ++s) {
        const float2* P = a.polar + (size_t)s * a.V * a.S;
        float dcv = 0.f;
        if (blockIdx.x == 0) {
            float acc = 0.f;
            for (int i = threadIdx.x; i < a.V; i += C::WG) acc += a.dc[(size_t)s * a.V + i];
            dcv = block_sum<C::WG>(acc, red) * a.dc_scale;
        }
        float2 v[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int o0 = off0[e];
            if (o0 >= 0) {
                const int o1 = off1[e];
                const float2* p0 = P + (o0 & kOffMask);
                const float2* p1 = P + (o1 & kOffMask);
                const float2 A0 = p0[0], A1 = p0[1], B0 = p1[0], B1 = p1[1];
                const float g = gr[e], f = fr[e];
                float2 u0 = make_float2(fmaf(g, A1.x - A0.x, A0.x), fmaf(g, A1.y - A0.y, A0.y));
                float2 u1 = make_float2(fmaf(g, B1.x - B0.x, B0.x), fmaf(g, B1.y - B0.y, B0.y));
                if (o0 & kConj) u0.y = -u0.y;
                if (o1 & kConj) u1.y = -u1.y;
                v[e] = make_float2(fmaf(f, u1.x - u0.x, u0.x), fmaf(f, u1.y - u0.y, u0.y));
            } else if (o0 == kDc) {
                v[e] = make_float2(dcv, 0.f);
            } else {
                v[e] = make_float2(0.f, 0.f);
            }
        }

        fft<LOGG, +1>(v, my, j, a.tw);

        if (live) {
            float2* D = a.grid + (size_t)s * a.N * (G / 2);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int y = j + e * T;
                const int p = (y + half_n) & (G - 1);
                if (p < a.N) D[((size_t)(p >> 3) * (G / 2) + col) * 8 + (p & 7)] = v[e];
            }
        }
    }
}

template <int LOGG>
static hipError_t launch_gather_t(const GatherArgs& a, hipStream_t st) {
    using C = GatherCfg<LOGG>;
    const int cols = C::G / 2;
    const int chunks = (a.batch + a.slices_per_block - 1) / a.slices_per_block;
    dim3 grid((cols + C::F - 1) / C::F, chunks);
    hipLaunchKernelGGL(k_gather_colifft<LOGG>, grid, dim3(C::WG), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gather_colifft(const bst_plan_s& p, const GatherArgs& a, hipStream_t st) {
    switch (p.logG) {
        case 4: return launch_gather_t<4>(a, st);
        case 5: return launch_gather_t<5>(a, st);
        case 6: return launch_gather_t<6>(a, st);
        case 7: return launch_gather_t<7>(a, st);
        case 8: return launch_gather_t<8>(a, st);
        case 9: return launch_gather_t<9>(a, st);
        case 10: return launch_gather_t<10>(a, st);
        case 11: return launch_gather_t<11>(a, st);
        case 12: return launch_gather_t<12>(a, st);
        case 13: return launch_gather_t<13>(a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bst
