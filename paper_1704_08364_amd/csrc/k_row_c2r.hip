// k_row_c2r.hip -- second half of step P6 (inverse DFT along k_x, complex to
// real) with P7/P8 (shift to the centre and crop to N columns) and the dk^2
// scale of the inverse Fourier integral (Section 2).
//
// Two output rows p, p+1 share one complex inverse FFT of length G:
//   W[k] = X_p[k] + i X_{p+1}[k] with the Hermitian extension
//   X[G-k] = conj X[k]; then x_p = Re w and x_{p+1} = Im w.
// As in the usual C2R convention the imaginary part of the k = 0 sample is
// ignored, and the k = G/2 sample is zero (no polar data reaches |k_x| = G/2).
// A block takes up to 8 rows, i.e. one contiguous [G/2][8] tile of the grid
// written by the column kernel, with the row pairs interleaved across lanes so
// that each wave's loads are contiguous.
#include "bst_internal.h"
#include "fft_lds.h"

namespace bst {

// extra float2 between the LDS regions of a block's row pairs
#ifndef BST_ROW_PAD
#define BST_ROW_PAD 8
#endif

// row pairs per block for G <= 4096 (one 8-row tile is 4 pairs)
#ifndef BST_ROW_PAIRS
#define BST_ROW_PAIRS 4
#endif

template <int LOGG>
struct RowCfg {
    static constexpr int G = 1 << LOGG;
    static constexpr int T = G / 16;
    static constexpr int F = G <= 4096 ? BST_ROW_PAIRS : (G == 8192 ? 2 : 1);  // row pairs per block
    static constexpr int WG = F * T;
};

template <int LOGG>
__global__ void __launch_bounds__(RowCfg<LOGG>::WG) k_row_c2r(RowArgs a) {
    using C = RowCfg<LOGG>;
    constexpr int G = C::G, T = C::T;
    // regions 8 float2 (16 banks) apart, so interleaved lanes of different row
    // pairs fall on different banks
    constexpr int STRIDE = FftShape<LOGG>::LDS + BST_ROW_PAD;
    __shared__ float2 lds[C::F * STRIDE];
    // thread t serves row pair t mod F: the lanes of a wave read F neighbouring
    // 16-byte pairs of each k, i.e. contiguous runs of the [G/2][8] tile
    const int fid = threadIdx.x % C::F;
    const int j = threadIdx.x / C::F;
    float2* my = lds + fid * STRIDE;
    const int row0 = blockIdx.x * (2 * C::F) + 2 * fid;
    const int s = blockIdx.y;
    const int sub = row0 & 7;
    const float4* tile = reinterpret_cast<const float4*>(
        a.grid + ((size_t)s * a.N + (size_t)(row0 >> 3) * 8) * a.GT);

    // all loads first, branch-free: k < G/2 reads k, k > G/2 reads G - k
    // (Hermitian extension), k = G/2 reads k = 0 and is replaced by zero
    float4 q[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int k = j + e * T;
        const int kk = k < G / 2 ? k : (k == G / 2 ? 0 : G - k);
        q[e] = tile[kk * 4 + (sub >> 1)];
    }
    float* o0 = (a.img_list ? a.img_list[s] : a.img + (size_t)s * a.N * a.N) + (size_t)row0 * a.N;
    float* o1 = o0 + a.N;

    float2 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int k = j + e * T;
        const bool mid = k == G / 2;
        // imaginary parts: dropped at k = 0 (C2R convention), conjugated for k > G/2
        const float sy = (k == 0 || mid) ? 0.f : (k < G / 2 ? 1.f : -1.f);
        const float2 x0 = make_float2(mid ? 0.f : q[e].x, sy * q[e].y);
        const float2 x1 = make_float2(mid ? 0.f : q[e].z, sy * q[e].w);
        v[e] = make_float2(x0.x - x1.y, x0.y + x1.x);
    }

    fft<LOGG, +1>(v, my, j, a.tw);

    const int half_n = a.N >> 1;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int x = j + e * T;
        const int c = (x + half_n) & (G - 1);
        if (c < a.N) {
            o0[c] = v[e].x * a.scale;
            o1[c] = v[e].y * a.scale;
        }
    }
}

template <int LOGG>
static hipError_t launch_row_t(const RowArgs& a, int batch, hipStream_t st) {
    using C = RowCfg<LOGG>;
    dim3 grid(a.N / (2 * C::F), batch);
    hipLaunchKernelGGL(k_row_c2r<LOGG>, grid, dim3(C::WG), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_row_c2r(const bst_plan_s& p, const RowArgs& a, int batch, hipStream_t st) {
    switch (p.logG) {
        case 4: return launch_row_t<4>(a, batch, st);
        case 5: return launch_row_t<5>(a, batch, st);
        case 6: return launch_row_t<6>(a, batch, st);
        case 7: return launch_row_t<7>(a, batch, st);
        case 8: return launch_row_t<8>(a, batch, st);
        case 9: return launch_row_t<9>(a, batch, st);
        case 10: return launch_row_t<10>(a, batch, st);
        case 11: return launch_row_t<11>(a, batch, st);
        case 12: return launch_row_t<12>(a, batch, st);
        case 13: return launch_row_t<13>(a, batch, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bst
