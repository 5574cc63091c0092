// k_gather_colifft.hip -- step P5 (polar -> Cartesian interpolation in the
// frequency domain, Section 2) fused with the first half of P6 (the inverse
// DFT along k_y) and the row part of P7/P8 (shift and crop).
//
// A block owns F neighbouring Cartesian columns k_x = a*dk (a in [0, G/2))
// and all G rows k_y = b*dk of each, b in FFT order; thread t works on column
// t mod F, so the lanes of a wave cover F neighbouring columns times 64/F
// neighbouring rows, and their polar reads fall on few cache lines (the same
// angle row, consecutive radii). Columns go to XCDs in contiguous ranges so
// neighbouring columns share an L2.
//
// Each thread keeps the interpolation coordinates of its E points (8 by
// default) in three registers each and reuses them for every slice of its
// chunk. They are exact
// to FP32 rounding although radius and angle indices reach a few thousand:
//   radius index r = |(a,b)| P_r/P_c from an FP64 square root;
//   angle index: an FP32 atan2 picks the interval [theta_j0, theta_j0+1), then
//   the offset inside it is atan2(cross, dot) of the point direction against
//   (cos theta_j0, sin theta_j0) from an FP64 table (cross and dot in FP64,
//   the small angle in FP32), so the fraction f carries no cancellation.
// Per slice, the column is gathered straight into the registers the FFT
// starts from, inverse-transformed along b, and only the N rows that survive
// the crop are written, to a grid laid out [N/8][G/2][8] (complex): the 8 rows
// of a tile and neighbouring columns form contiguous runs, and the row kernel
// reads each 8-row tile contiguously.
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

// threads per block of the gather kernel (the columns per block follow from it)
#ifndef BST_GATHER_THREADS
#define BST_GATHER_THREADS 512
#endif

// waves per SIMD the register allocation must leave room for
#ifndef BST_GATHER_WAVES
#define BST_GATHER_WAVES 4
#endif

// two adjacent complex samples; 8-byte aligned, read with one 16-byte load
struct __attribute__((aligned(8))) Pair8 {
    float x0, y0, x1, y1;
};

// point code: bits 0-13 j0, 14-26 m0, 27 conjugate the j0 samples, 28 conjugate the j1 samples
constexpr unsigned kCodeZero = 0xFFFFFFFFu;
constexpr unsigned kCodeDc = 0xFFFFFFFEu;
constexpr unsigned kConj0 = 1u << 27;
constexpr unsigned kConj1 = 1u << 28;
constexpr unsigned kWrapShift = 29;  // bit 29: the j1 neighbour wraps to angle 0

template <int LOGG, int EV>
struct GatherCfg {
    static constexpr int G = 1 << LOGG;
    static constexpr int E = EV;
    static constexpr int T = G / E;
    static constexpr int MAXT = BST_GATHER_THREADS > T ? BST_GATHER_THREADS : T;
    static constexpr int FL = 16384 / G;                 // LDS: about 140 KB of transforms
    static constexpr int F1 = FL < G / 2 ? FL : G / 2;   // no more columns than exist
    static constexpr int F2 = MAXT / T;
    static constexpr int F = F1 < F2 ? F1 : F2;          // columns per block
    static constexpr int WG = F * T;
    // transform stride in LDS: padded length plus 8 float2, so that F regions
    // start 16 banks apart and lanes of different columns do not collide
    static constexpr int STRIDE = FftShape<LOGG>::LDS + 8;
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

// Interpolation coordinates of Cartesian point (col, bs); bs signed.
__device__ __forceinline__ unsigned point_code(int col, int bs, const GatherArgs& a, float& f_out, float& g_out) {
    f_out = 0.f;
    g_out = 0.f;
    if (col == 0 && bs == 0) return kCodeDc;
    const double r = sqrt((double)(col * col + bs * bs)) * a.rscale;
    if (r >= (double)a.Mh) return kCodeZero;
    const double mf = floor(r);
    g_out = (float)(r - mf);
    const unsigned m0 = (unsigned)mf;

    // direction of the point on [0, pi): (x, y) with y >= 0
    const bool lower = bs < 0;
    const int x = lower ? -col : col;
    const int y = lower ? -bs : bs;
    const float th = atan2f((float)y, (float)x);
    int j0 = (int)floorf(th * a.vpi_f);
    j0 = j0 < 0 ? 0 : (j0 >= a.V ? a.V - 1 : j0);
    const double2 cs = a.ang[j0];
    const double cross = (double)y * cs.x - (double)x * cs.y;
    const double dot = (double)x * cs.x + (double)y * cs.y;
    float f = atan2f((float)cross, (float)dot) * a.vpi_f;
    if (f < 0.f) {
        if (j0 > 0) { j0 -= 1; f += 1.f; } else { f = 0.f; }
    } else if (f >= 1.f) {
        if (j0 < a.V - 1) { j0 += 1; f -= 1.f; } else { f = 1.f; }
    }
    f_out = f;
    const bool wrap = (j0 + 1 == a.V);
    unsigned code = (unsigned)j0 | (m0 << 14);
    if (lower) code |= kConj0;
    if (lower != wrap) code |= kConj1;
    if (wrap) code |= 1u << kWrapShift;
    return code;
}

template <int LOGG, int EV>
__global__ void __launch_bounds__((GatherCfg<LOGG, EV>::WG))
__attribute__((amdgpu_waves_per_eu(EV == 8 ? BST_GATHER_WAVES : 1, 8))) k_gather_colifft(GatherArgs a) {
    using C = GatherCfg<LOGG, EV>;
    constexpr int G = C::G, T = C::T, F = C::F, E = C::E;
    __shared__ float2 lds[F * C::STRIDE];
    __shared__ float red[(C::WG + 63) / 64];
    const int fid = threadIdx.x % F;
    const int j = threadIdx.x / F;
    float2* my = lds + fid * C::STRIDE;
    const int lblock = xcd_contiguous(blockIdx.x, gridDim.x);
    const int col = lblock * F + fid;
    const bool live = col < G / 2;

    // Coordinates: computed in a rolled loop (one copy of the trigonometry in
    // registers), staged through the still unused transform LDS in chunks of
    // 4 points, then held in registers for the whole chunk of slices.
    constexpr int CH = 4;
    unsigned code[E];
    float fr[E], gr[E];
    static_assert(C::F * C::STRIDE * 2 >= C::WG * CH * 3, "coordinate staging needs LDS");
    unsigned* st_code = reinterpret_cast<unsigned*>(lds);
    float* st_f = reinterpret_cast<float*>(lds) + C::WG * CH;
    float* st_g = st_f + C::WG * CH;
#pragma unroll
    for (int c0 = 0; c0 < E; c0 += CH) {
#pragma unroll 1
        for (int h = 0; h < CH; ++h) {
            const int b = j + (c0 + h) * T;
            const int bs = b < G / 2 ? b : b - G;
            float f = 0.f, g = 0.f;
            const unsigned c = live ? point_code(col, bs, a, f, g) : kCodeZero;
            st_code[h * C::WG + threadIdx.x] = c;
            st_f[h * C::WG + threadIdx.x] = f;
            st_g[h * C::WG + threadIdx.x] = g;
        }
#pragma unroll
        for (int h = 0; h < CH; ++h) {
            code[c0 + h] = st_code[h * C::WG + threadIdx.x];
            fr[c0 + h] = st_f[h * C::WG + threadIdx.x];
            gr[c0 + h] = st_g[h * C::WG + threadIdx.x];
        }
    }
    __syncthreads();  // the transform reuses this LDS

    const int s_begin = blockIdx.y * a.slices_per_block;
    const int s_end = min(a.batch, s_begin + a.slices_per_block);
    const int half_n = a.N >> 1;
    const int S = a.S;
    for (int s = s_begin; s < s_end; ++s) {
        const float2* P = a.polar + (size_t)s * a.V * S;
        float dcv = 0.f;
        if (lblock == 0) {
            float acc = 0.f;
            for (int i = threadIdx.x; i < a.V; i += C::WG) acc += a.dc[(size_t)s * a.V + i];
            dcv = block_sum<C::WG>(acc, red) * a.dc_scale;
        }
        float2 v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const unsigned c = code[e];
            if (c < kCodeDc) {
                const int j0 = c & 0x3FFF;
                const int m0 = (c >> 14) & 0x1FFF;
                const int o0 = j0 * S + m0;
                const int o1 = ((c >> kWrapShift) & 1u) ? m0 : o0 + S;
                // samples m0 and m0+1 of a row are adjacent: one 16-byte load each
                const Pair8 pa = *reinterpret_cast<const Pair8*>(P + o0);
                const Pair8 pb = *reinterpret_cast<const Pair8*>(P + o1);
                const float g = gr[e], f = fr[e];
                float2 u0 = make_float2(fmaf(g, pa.x1 - pa.x0, pa.x0), fmaf(g, pa.y1 - pa.y0, pa.y0));
                float2 u1 = make_float2(fmaf(g, pb.x1 - pb.x0, pb.x0), fmaf(g, pb.y1 - pb.y0, pb.y0));
                if (c & kConj0) u0.y = -u0.y;
                if (c & kConj1) u1.y = -u1.y;
                v[e] = make_float2(fmaf(f, u1.x - u0.x, u0.x), fmaf(f, u1.y - u0.y, u0.y));
            } else if (c == kCodeDc) {
                v[e] = make_float2(dcv, 0.f);
            } else {
                v[e] = make_float2(0.f, 0.f);
            }
        }

        fft<LOGG, +1, E>(v, my, j, a.tw);

        if (live) {
            float2* D = a.grid + (size_t)s * a.N * (G / 2);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int y = j + e * T;
                const int p = (y + half_n) & (G - 1);
                if (p < a.N) D[((size_t)(p >> 3) * (G / 2) + col) * 8 + (p & 7)] = v[e];
            }
        }
    }
}

template <int LOGG, int EV>
static hipError_t launch_gather_t(const GatherArgs& a, hipStream_t st) {
    using C = GatherCfg<LOGG, EV>;
    const int cols = C::G / 2;
    const int chunks = (a.batch + a.slices_per_block - 1) / a.slices_per_block;
    dim3 grid((cols + C::F - 1) / C::F, chunks);
    hipLaunchKernelGGL((k_gather_colifft<LOGG, EV>), grid, dim3(C::WG), 0, st, a);
    return hipGetLastError();
}

template <int LOGG>
static hipError_t launch_gather_e(const GatherArgs& a, int e, hipStream_t st) {
    if (e == 16) return launch_gather_t<LOGG, 16>(a, st);
    return launch_gather_t<LOGG, 8>(a, st);
}

hipError_t launch_gather_colifft(const bst_plan_s& p, const GatherArgs& a, hipStream_t st) {
    const int e = p.gather_e;
    switch (p.logG) {
        case 4: return launch_gather_e<4>(a, e, st);
        case 5: return launch_gather_e<5>(a, e, st);
        case 6: return launch_gather_e<6>(a, e, st);
        case 7: return launch_gather_e<7>(a, e, st);
        case 8: return launch_gather_e<8>(a, e, st);
        case 9: return launch_gather_e<9>(a, e, st);
        case 10: return launch_gather_e<10>(a, e, st);
        case 11: return launch_gather_e<11>(a, e, st);
        case 12: return launch_gather_e<12>(a, e, st);
        case 13: return launch_gather_e<13>(a, e, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bst
