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
#include "bst_check.h"
#include "monopole.h"

namespace bst {

// most row-pair groups (8-row tiles) a block walks, for G <= 4096
#ifndef BST_ROW_TILES
#define BST_ROW_TILES 16
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
    static constexpr int MAX_TILES = G <= 4096 ? BST_ROW_TILES : 1;  // row-pair groups per block, at most
    static_assert(T * 16 == G, "16 values per thread");
};

// MONO: adds m b_phi(u), the closed-form backprojection of the subtracted
// monopole, to every output pixel.
// Block (bx, s): row-pair groups bx * tiles .. of slice s.
template <int LOGG, bool MONO>
__device__ __forceinline__ void row_body(const RowArgs& a, int bx, int s) {
    using C = RowCfg<LOGG>;
    constexpr int G = C::G, T = C::T;
    // one LDS region of G float2 per row pair, the pairs' lanes interleaved
    __shared__ __attribute__((aligned(16))) float2 lds[C::F * G];
    // thread t serves row pair t mod F: the lanes of a wave read F neighbouring
    // 16-byte pairs of each k, i.e. contiguous runs of the [G/2][8] tile
    const int fid = threadIdx.x % C::F;
    const int j = threadIdx.x / C::F;
    const unsigned my_off = (unsigned)(fid * G) * 8u;
    const int xm = region_xor<LOGG, C::F>(fid);
    const int groups = a.N / (2 * C::F);             // row-pair groups (tiles) per slice
    const int g0 = bx * a.tiles;
    float* const img_s = a.img_list ? a.img_list[s] : a.img + (size_t)s * a.N * a.N;
    const FftTwiddles<LOGG, +1, 16> tw(j, a.tw);
    float mamp = 0.f;
    if constexpr (MONO) {
        const float inv = a.Vs ? a.mono_inv * (float)a.V / (float)a.Vs[s] : a.mono_inv;
        mamp = monopole_mass(a.mono_part, s, inv) * a.mono_amp;
    }

    // Thread j's slots e < 8 are k = j + e*T < G/2: the block reads every
    // stored column once (all loads first, no branch between them) and puts
    // it in LDS, where the Hermitian extension k > G/2 (the conjugate of
    // column G - k) is read back; k = G/2 is zero. A block walks TILES
    // groups, the next group's reads in flight during the current group's
    // transform.
    auto load = [&](int grp, float4 (&q)[8]) {
        const int row0 = (grp < groups ? grp : 0) * (2 * C::F) + 2 * fid;
        const float4* tile = reinterpret_cast<const float4*>(
            a.grid + ((size_t)s * a.N + (size_t)(row0 >> 3) * 8) * a.GT);
#pragma unroll
        for (int e = 0; e < 8; ++e) q[e] = tile[BST_IDX((j + e * T) * 4 + ((row0 & 7) >> 1), 4 * a.GT, 0)];
    };
    float4 q[8];
    load(g0, q);
#pragma unroll 1
    for (int it = 0; it < a.tiles; ++it) {
        const int grp = g0 + it;
        int jv = j;
        asm volatile("" : "+v"(jv));
        float4* stage = reinterpret_cast<float4*>(lds);  // [G/2][F] of the group's row pairs
#pragma unroll
        for (int e = 0; e < 8; ++e) stage[(jv + e * T) * C::F + fid] = q[e];
        __syncthreads();

        float2 v[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int k = jv + e * T;
            const bool lo = e < 8;
            const int kk = G - k;                     // mirrored column for k > G/2
            const float4 m = lo ? q[e] : stage[(kk & (G / 2 - 1)) * C::F + fid];
            const bool mid = k == G / 2;
            // imaginary parts: dropped at k = 0 (C2R convention), conjugated for k > G/2
            const float sy = (k == 0 || mid) ? 0.f : (lo ? 1.f : -1.f);
            const float2 x0 = make_float2(mid ? 0.f : m.x, sy * m.y);
            const float2 x1 = make_float2(mid ? 0.f : m.z, sy * m.w);
            v[e] = make_float2(x0.x - x1.y, x0.y + x1.x);
        }
        __syncthreads();  // the transform overwrites the staged columns
        if (it + 1 < a.tiles) load(grp + 1, q);

        FftTwiddles<LOGG, +1, 16> twl = tw;
        twl.pin();
        fft<LOGG, +1>(v, lds, my_off, jv, twl, xm);

        if (grp < groups) {
            const int row0 = BST_IDX(grp * (2 * C::F) + 2 * fid, a.N - 1, 1);
            float* o0 = img_s + (size_t)row0 * a.N;
            float* o1 = o0 + a.N;
            const int half_n = a.N >> 1;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int x = jv + e * T;
                const int c = (x + half_n) & (G - 1);
                if (c < a.N) {
                    float b0 = v[e].x * a.scale, b1 = v[e].y * a.scale;
                    if constexpr (MONO) {
                        // pixel offsets from the centre: exact in float (|.|^2 <= 2^23)
                        const float dx = (float)(c - half_n), dy = (float)(row0 - half_n);
                        const float r0 = dx * dx + dy * dy;
                        const float r1 = r0 + 2.f * dy + 1.f;
                        b0 += mamp * scaled_bessel_i0(a.mono_rho_px * r0);
                        b1 += mamp * scaled_bessel_i0(a.mono_rho_px * r1);
                    }
                    o0[BST_IDX(c, a.N, 2)] = b0;
                    o1[BST_IDX(c, a.N, 2)] = b1;
                }
            }
        }
    }
}

template <int LOGG, bool MONO>
__global__ void __launch_bounds__(RowCfg<LOGG>::WG) k_row_c2r(RowArgs a) {
    row_body<LOGG, MONO>(a, blockIdx.x, blockIdx.y);
}

// Persistent launch of uneven batches: every block walks the work list
// (slice, block) in steps of the grid.
template <int LOGG, bool MONO>
__global__ void __launch_bounds__(RowCfg<LOGG>::WG) k_row_items(RowArgs a) {
    const int local = xcd_contiguous(blockIdx.x, gridDim.x);
    for (int base = 0; base < a.n_items; base += gridDim.x) {
        const int it = base + local;
        if (it >= a.n_items) break;
        const int2 w = a.items[it];
        __syncthreads();  // the previous item's LDS reads are done
        row_body<LOGG, MONO>(a, w.y, w.x);
    }
}

template <int LOGG>
static hipError_t launch_row_t(const RowArgs& a0, int batch, hipStream_t st) {
    using C = RowCfg<LOGG>;
    RowArgs a = a0;
    const int groups = a.N / (2 * C::F);
    // as many groups per block as keep about four blocks per compute unit
    constexpr int kTargetBlocks = 1024;
    int tiles = (int)(((long long)groups * batch) / kTargetBlocks);
    tiles = tiles < 1 ? 1 : (tiles > C::MAX_TILES ? C::MAX_TILES : tiles);
    a.tiles = tiles;
    dim3 grid((groups + tiles - 1) / tiles, batch);
    if (a.mono_part) hipLaunchKernelGGL((k_row_c2r<LOGG, true>), grid, dim3(C::WG), 0, st, a);
    else hipLaunchKernelGGL((k_row_c2r<LOGG, false>), grid, dim3(C::WG), 0, st, a);
    return hipGetLastError();
}

template <int LOGG>
static hipError_t launch_row_items_t(const RowArgs& a, int blocks, hipStream_t st) {
    using C = RowCfg<LOGG>;
    if (a.tiles < 1 || a.tiles > C::MAX_TILES) return hipErrorInvalidValue;
    if (a.mono_part) hipLaunchKernelGGL((k_row_items<LOGG, true>), dim3(blocks), dim3(C::WG), 0, st, a);
    else hipLaunchKernelGGL((k_row_items<LOGG, false>), dim3(blocks), dim3(C::WG), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_row_items(const bst_plan_s& p, const RowArgs& a, int blocks, hipStream_t st) {
    switch (p.logG) {
        case 4: return launch_row_items_t<4>(a, blocks, st);
        case 5: return launch_row_items_t<5>(a, blocks, st);
        case 6: return launch_row_items_t<6>(a, blocks, st);
        case 7: return launch_row_items_t<7>(a, blocks, st);
        case 8: return launch_row_items_t<8>(a, blocks, st);
        case 9: return launch_row_items_t<9>(a, blocks, st);
        case 10: return launch_row_items_t<10>(a, blocks, st);
        case 11: return launch_row_items_t<11>(a, blocks, st);
        case 12: return launch_row_items_t<12>(a, blocks, st);
        case 13: return launch_row_items_t<13>(a, blocks, st);
        default: return hipErrorInvalidValue;
    }
}

template <int LOGG>
static int row_blocks_t(int N, int tiles) {
    using C = RowCfg<LOGG>;
    const int groups = N / (2 * C::F);
    tiles = tiles < 1 ? 1 : (tiles > C::MAX_TILES ? C::MAX_TILES : tiles);
    return (groups + tiles - 1) / tiles;
}

int row_max_tiles(const bst_plan_s& p) {
    switch (p.logG) {
        case 4: return RowCfg<4>::MAX_TILES;
        case 5: return RowCfg<5>::MAX_TILES;
        case 6: return RowCfg<6>::MAX_TILES;
        case 7: return RowCfg<7>::MAX_TILES;
        case 8: return RowCfg<8>::MAX_TILES;
        case 9: return RowCfg<9>::MAX_TILES;
        case 10: return RowCfg<10>::MAX_TILES;
        case 11: return RowCfg<11>::MAX_TILES;
        case 12: return RowCfg<12>::MAX_TILES;
        case 13: return RowCfg<13>::MAX_TILES;
        default: return 1;
    }
}

int row_blocks_per_slice(const bst_plan_s& p, int tiles) {
    switch (p.logG) {
        case 4: return row_blocks_t<4>(p.N, tiles);
        case 5: return row_blocks_t<5>(p.N, tiles);
        case 6: return row_blocks_t<6>(p.N, tiles);
        case 7: return row_blocks_t<7>(p.N, tiles);
        case 8: return row_blocks_t<8>(p.N, tiles);
        case 9: return row_blocks_t<9>(p.N, tiles);
        case 10: return row_blocks_t<10>(p.N, tiles);
        case 11: return row_blocks_t<11>(p.N, tiles);
        case 12: return row_blocks_t<12>(p.N, tiles);
        case 13: return row_blocks_t<13>(p.N, tiles);
        default: return 0;
    }
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

BST_CHECK_MODULE(row)
