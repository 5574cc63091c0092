// k_project.hip -- the projector R of bst_project: the exact adjoint of the
// BST backprojection (Section 2, steps P8 .. P1 transposed one by one).
//
//   k_proj_rows    transpose of the row C2R + crop + dk^2: image rows are
//                  zero-embedded at (q - N/2) mod G, forward-transformed two
//                  rows per complex FFT, split, and scaled by dk^2 * c_a
//                  (c_0 = 1, c_a = 2 otherwise: the C2R counts interior
//                  columns twice); written to 8-row tiles [N/8][G/2][8].
//   k_proj_cols    transpose of the column inverse DFT + crop: each column's N
//                  rows are zero-embedded at (p - N/2) mod G and forward
//                  transformed; the full half-plane spectra are written
//                  column-major with 16 slices interleaved per point
//                  ([batch/16][G/2 * G][16]).
//   k_proj_gather  transpose of the bilinear polar -> Cartesian gather: every
//                  polar sample sums, in a fixed order, the Cartesian values
//                  whose stencil contains it (CSR lists built once per plan,
//                  weight and conjugation per entry). No atomics, so the result
//                  is bitwise reproducible. Each list is read once for up to 16
//                  slices; blocks take 16 x 16 tiles of (angle, radius),
//                  spread XCD-contiguously.
//   k_proj_polar   transpose of P4..P1: the conjugate of the complex radial
//                  weight dt*K[m]*A*phase (plus the origin rule's share
//                  on m = 0), the transpose of the real DFT as the inverse FFT
//                  of the Hermitian extension (two projections per complex
//                  FFT), crop of the zero padding, taper, and the factor
//                  d^2 / (dt w_j) (w_j = pi/V for uniform angles, else half
//                  the neighbour gap) that makes R the weighted-inner-product
//                  adjoint of B.
#include "bst_internal.h"
#include "bst_check.h"
#include "fft_lds.h"

namespace bst {

template <int LOGG>
struct ProjRowCfg {
    static constexpr int G = 1 << LOGG;
    static constexpr int T = G / 16;
    static constexpr int F = G <= 4096 ? 4 : 2;   // row pairs per block
    static constexpr int WG = F * T;
};

template <int LOGG>
__global__ void __launch_bounds__(ProjRowCfg<LOGG>::WG) k_proj_rows(ProjRowArgs a) {
    using C = ProjRowCfg<LOGG>;
    constexpr int G = C::G, T = C::T;
    __shared__ float2 lds[C::F * G];  // one region per row pair, the pairs' lanes interleaved
    const int fid = threadIdx.x % C::F;
    const int j = threadIdx.x / C::F;
    const unsigned my_off = (unsigned)(fid * G) * 8u;
    const int xm = region_xor<LOGG, C::F>(fid);
    const int row0 = blockIdx.x * (2 * C::F) + 2 * fid;
    const int s = blockIdx.y;
    const float* r0 = a.img + ((size_t)s * a.N + row0) * a.N;
    const float* r1 = r0 + a.N;
    const int half_n = a.N >> 1;

    // loads first, branch-free: columns outside the crop read column 0 and
    // are replaced by zero
    float x0[16], x1[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int q = (j + e * T + half_n) & (G - 1);
        const int qq = q < a.N ? q : 0;
        x0[e] = r0[qq];
        x1[e] = r1[qq];
    }
    float2 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int q = (j + e * T + half_n) & (G - 1);
        v[e] = q < a.N ? make_float2(x0[e], x1[e]) : make_float2(0.f, 0.f);
    }
    fft<LOGG, -1>(v, lds, my_off, j, a.tw, xm);
    const unsigned pj = lds_byte(my_off, lds_swz<16>(j), xm);
#pragma unroll
    for (int e = 0; e < 16; ++e) lds_at(lds, pj ^ swz_bytes<16>(e * T)) = v[e];
    __syncthreads();

    float4* tile = reinterpret_cast<float4*>(a.grid + ((size_t)s * a.N + (size_t)(row0 >> 3) * 8) * (G / 2));
    const int sub = row0 & 7;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = j + e * T;  // 0 .. G/2-1
        const float2 z = lds_at(lds, lds_byte(my_off, lds_swz<16>(k), xm));
        const float2 zc = lds_at(lds, lds_byte(my_off, lds_swz<16>((G - k) & (G - 1)), xm));
        const float c = (k == 0 ? 0.5f : 1.0f) * a.scale;  // dk^2 * c_a / 2
        tile[k * 4 + (sub >> 1)] = make_float4(c * (z.x + zc.x), c * (z.y - zc.y),
                                               c * (z.y + zc.y), -c * (z.x - zc.x));
    }
}

template <int LOGG>
struct ProjColCfg {
    static constexpr int G = 1 << LOGG;
    static constexpr int T = G / 16;
    static constexpr int SL0 = T >= 512 ? 1 : 512 / T;
    static constexpr int SL = SL0 > kProjInterleave ? kProjInterleave : SL0;  // slices per round
    static constexpr int ROUNDS = kProjInterleave / SL;
    static constexpr int WG = SL * T;
};

// Column transform of one slot of the group (zeros past the batch).
template <int LOGG>
__device__ __forceinline__ void proj_col_transform(const ProjColArgs& a, int grp, int col, int slot, int j,
                                                   float2* lds, unsigned off, int xm, float2 (&v)[16]) {
    using C = ProjColCfg<LOGG>;
    constexpr int G = C::G, T = C::T;
    const int s = grp * kProjInterleave + slot;
    const bool live = s < a.batch;
    const int half_n = a.N >> 1;
    // loads first, branch-free: rows outside the crop (and slots past the
    // batch) read a valid element and are replaced by zero
    const float2* D = a.grid + (size_t)(live ? s : 0) * a.N * (G / 2);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int p = (j + e * T + half_n) & (G - 1);
        const int pp = p < a.N ? p : 0;
        v[e] = D[((size_t)(pp >> 3) * (G / 2) + col) * 8 + (pp & 7)];
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int p = (j + e * T + half_n) & (G - 1);
        if (!(live && p < a.N)) v[e] = make_float2(0.f, 0.f);
    }
    fft<LOGG, -1>(v, lds, off, j, a.tw, xm);
}

// One block per Cartesian column a and group of kProjInterleave slices: the
// group's slices are transformed SL at a time, and each result is stored
// straight into the interleaved layout [group][a * G + b][slot] that the
// transposed gather reads. Where the group takes two or more rounds, each
// thread takes two adjacent slots per pass, so the SL threads that hold
// point b write 2 * SL adjacent slots of one 128-byte line, and the block
// completes each of its lines within a few passes, so the partial writes
// meet in L2 (small grids transform the whole group in one round). Logical
// blocks are spread XCD-contiguously, so neighbouring columns (which share
// the input tiles' lines) share an L2. Slots past the batch are written as
// zeros.
template <int LOGG>
__global__ void __launch_bounds__(ProjColCfg<LOGG>::WG) k_proj_cols(ProjColArgs a) {
    using C = ProjColCfg<LOGG>;
    constexpr int G = C::G, T = C::T;
    __shared__ float2 lds[C::SL * G];  // one region per slice, the slices' lanes interleaved
    const int unit = xcd_contiguous(blockIdx.x, gridDim.x);
    if (unit >= a.units) return;  // whole block, before any barrier
    const int grp = unit / (G / 2), col = unit % (G / 2);
    const int fid = threadIdx.x % C::SL;
    const int j0 = threadIdx.x / C::SL;
    const unsigned my_off = (unsigned)(fid * G) * 8u;
    const int xm = region_xor<LOGG, C::SL>(fid);
    float2* out = a.cart8 + ((size_t)grp * (G / 2) * G + (size_t)col * G) * kProjInterleave;
    if constexpr (C::ROUNDS >= 2) {
        // two rounds per pass: each thread transforms two adjacent slots and
        // stores them as one 16-byte write
#pragma unroll 1
        for (int r = 0; r < C::ROUNDS; r += 2) {
            // addresses are re-derived each pass from an opaque copy of the
            // thread index rather than held in registers across passes
            int j = j0;
            asm volatile("" : "+v"(j));
            const int slot = r * C::SL + 2 * fid;
            float2 va[16], vb[16];
            proj_col_transform<LOGG>(a, grp, col, slot, j, lds, my_off, xm, va);
            __syncthreads();
            proj_col_transform<LOGG>(a, grp, col, slot + 1, j, lds, my_off, xm, vb);
            float4* o4 = reinterpret_cast<float4*>(out);
#pragma unroll
            for (int e = 0; e < 16; ++e)
                o4[BST_IDX(((size_t)(j + e * T) * kProjInterleave + slot) / 2, (size_t)G * kProjInterleave / 2, 1)] =
                    make_float4(va[e].x, va[e].y, vb[e].x, vb[e].y);
            __syncthreads();
        }
    } else {
        const int slot = fid;
        float2 v[16];
        proj_col_transform<LOGG>(a, grp, col, slot, j0, lds, my_off, xm, v);
#pragma unroll
        for (int e = 0; e < 16; ++e)
            out[BST_IDX((size_t)(j0 + e * T) * kProjInterleave + slot, (size_t)G * kProjInterleave, 1)] = v[e];
    }
}

// Transposed gather: each polar sample and group of kProjInterleave slices
// sums the sample's list of Cartesian points (weights and conjugation flags
// from the plan), in list order. Eight lanes share a sample, each summing two
// of the group's slices, so that one 16-byte read per lane covers a list
// entry's whole 128-byte line (the interleaved slices of one Cartesian point)
// and every read of a wave is a full line. A block of 256 threads takes a
// tile of kProjTileAngles x kProjTileRadii samples, 32 at a time, and the
// tiles, radius-fastest, are spread XCD-contiguously: the samples of
// neighbouring angles and radii share stencil points, so a tile and its
// successors on one XCD find them in that XCD's L2.
constexpr int kProjTileAngles = 16, kProjTileRadii = 16;
constexpr int kProjLanes = kProjInterleave / 2;  // lanes per sample, two slices each
constexpr int kProjGatherThreads = 256;
constexpr int kProjBurst = 4;  // list entries whose reads are issued together
__global__ void __launch_bounds__(kProjGatherThreads) k_proj_gather(ProjGatherArgs a) {
    const int tiles_m = (a.half_m + kProjTileRadii - 1) / kProjTileRadii;
    const int tile = xcd_contiguous(blockIdx.x, gridDim.x);
    const int m_base = (tile % tiles_m) * kProjTileRadii;
    const int j_base = (tile / tiles_m) * kProjTileAngles;
    const int p = threadIdx.x % kProjLanes;  // this lane's slices: 2p, 2p + 1 of the group
    const int sa = blockIdx.y * kProjInterleave + 2 * p, sb = sa + 1;
    const float4* base = reinterpret_cast<const float4*>(a.cart + (size_t)blockIdx.y * a.cart_stride * kProjInterleave);
    constexpr int kPerRound = kProjGatherThreads / kProjLanes;
    for (int r = threadIdx.x / kProjLanes; r < kProjTileAngles * kProjTileRadii; r += kPerRound) {
        const int m = m_base + r % kProjTileRadii;
        const int j = j_base + r / kProjTileRadii;
        if (m >= a.half_m || j * a.half_m >= a.samples) continue;
        const int idx = j * a.half_m + m;
        float2 acc0 = make_float2(0.f, 0.f), acc1 = make_float2(0.f, 0.f);
        const int e1 = a.off[idx + 1];
        // the list kProjBurst entries at a time: all entry reads, then all
        // their data reads, then the sums in list order (an entry past the
        // end re-reads the last one and is not added)
        for (int e = a.off[idx]; e < e1; e += kProjBurst) {
            uint2 en[kProjBurst];
#pragma unroll
            for (int u = 0; u < kProjBurst; ++u) en[u] = a.ent[min(e + u, e1 - 1)];
            float4 q[kProjBurst];
#pragma unroll
            for (int u = 0; u < kProjBurst; ++u) {
                const size_t pidx = BST_IDX((size_t)(en[u].x & 0x7FFFFFFFu), (size_t)a.cart_stride, 0);
                q[u] = base[pidx * kProjLanes + p];
            }
#pragma unroll
            for (int u = 0; u < kProjBurst; ++u) {
                if (e + u < e1) {
                    const float w = __uint_as_float(en[u].y);
                    const float wy = (en[u].x >> 31) != 0u ? -w : w;  // conjugation folded into the weight
                    acc0.x = fmaf(w, q[u].x, acc0.x);
                    acc0.y = fmaf(wy, q[u].y, acc0.y);
                    acc1.x = fmaf(w, q[u].z, acc1.x);
                    acc1.y = fmaf(wy, q[u].w, acc1.y);
                }
            }
        }
        if (sa < a.batch) a.polar[(size_t)sa * a.samples + idx] = acc0;
        if (sb < a.batch) a.polar[(size_t)sb * a.samples + idx] = acc1;
    }
}

template <int LOGM>
struct ProjPolarCfg {
    static constexpr int M = 1 << LOGM;
    static constexpr int T = M / 16;
    static constexpr int F = T >= 256 ? 1 : 256 / T;   // projection pairs per block
    static constexpr int WG = F * T;
};

template <int LOGM>
__global__ void __launch_bounds__(ProjPolarCfg<LOGM>::WG)
__attribute__((amdgpu_waves_per_eu(4, 8))) k_proj_polar(ProjPolarArgs a) {
    using C = ProjPolarCfg<LOGM>;
    constexpr int M = C::M, T = C::T;
    __shared__ float2 lds[C::F * M];
    const int fid = threadIdx.x / T;
    const int j = threadIdx.x - fid * T;
    const unsigned my_off = (unsigned)(fid * M) * 8u;  // this pair's LDS region
    const int my_xm = contiguous_xor<LOGM, T>(fid);
    const int pair = blockIdx.x * C::F + fid;
    const int s = blockIdx.y;
    const int ja = 2 * pair, jb = 2 * pair + 1;
    const bool va = ja < a.V, vb = jb < a.V;
    const float2* PA = a.polar + ((size_t)s * a.V + (va ? ja : 0)) * (M / 2);
    const float2* PB = a.polar + ((size_t)s * a.V + (vb ? jb : 0)) * (M / 2);
    const float dct =
        a.dc_dt * a.cart[(size_t)(s / kProjInterleave) * a.cart_stride * kProjInterleave + s % kProjInterleave].x;

    // loads first, branch-free: sample m = |k| of both projections and its
    // weight; k = M/2 reads m = 0 and is replaced by zero
    float2 xa[16], xb[16], wk[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int k = j + e * T;
        const int m = k < M / 2 ? k : (k == M / 2 ? 0 : M - k);
        xa[e] = PA[m];
        xb[e] = PB[m];
        wk[e] = a.kc[m];
    }
    float2 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int k = j + e * T;
        const bool up = k < M / 2;
        float2 ha, hb;
        if (k == 0) {
            // the weight is real at sigma = 0 (phase 1); the origin rule adds dct
            ha = make_float2(wk[e].x * xa[e].x + dct, 0.f);
            hb = make_float2(wk[e].x * xb[e].x + dct, 0.f);
        } else {
            const float2 w = make_float2(0.5f * wk[e].x, -0.5f * wk[e].y);  // conj(weight)/2
            const float2 ya = cmul(xa[e], w), yb = cmul(xb[e], w);
            ha = up ? ya : make_float2(ya.x, -ya.y);
            hb = up ? yb : make_float2(yb.x, -yb.y);
        }
        if (k == M / 2 || !va) ha = make_float2(0.f, 0.f);
        if (k == M / 2 || !vb) hb = make_float2(0.f, 0.f);
        v[e] = make_float2(ha.x - hb.y, ha.y + hb.x);
    }
    fft<LOGM, +1>(v, lds, my_off, j, a.tw, my_xm);

    const int h = a.n >> 1;
    float* oa = a.sino + ((size_t)s * a.V + ja) * a.n;
    float* ob = oa + a.n;
    const float sa = a.row_scale[va ? ja : 0], sb = a.row_scale[vb ? jb : 0];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int x = j + e * T;
        const int i = (x < h) ? x + h : ((x >= M - h) ? x - M + h : -1);
        if (i >= 0) {
            const float w = a.taper[i];
            if (va) oa[i] = (w * sa) * v[e].x;
            if (vb) ob[i] = (w * sb) * v[e].y;
        }
    }
}

#define BST_SWITCH_LOG(L, FN, ...)                  \
    switch (L) {                                    \
        case 4: return FN<4>(__VA_ARGS__);          \
        case 5: return FN<5>(__VA_ARGS__);          \
        case 6: return FN<6>(__VA_ARGS__);          \
        case 7: return FN<7>(__VA_ARGS__);          \
        case 8: return FN<8>(__VA_ARGS__);          \
        case 9: return FN<9>(__VA_ARGS__);          \
        case 10: return FN<10>(__VA_ARGS__);        \
        case 11: return FN<11>(__VA_ARGS__);        \
        case 12: return FN<12>(__VA_ARGS__);        \
        case 13: return FN<13>(__VA_ARGS__);        \
        default: return hipErrorInvalidValue;       \
    }

template <int LOGG>
static hipError_t proj_rows_t(const ProjRowArgs& a, int batch, hipStream_t st) {
    using C = ProjRowCfg<LOGG>;
    hipLaunchKernelGGL(k_proj_rows<LOGG>, dim3(a.N / (2 * C::F), batch), dim3(C::WG), 0, st, a);
    return hipGetLastError();
}
template <int LOGG>
static hipError_t proj_cols_t(const ProjColArgs& a, int batch, hipStream_t st) {
    using C = ProjColCfg<LOGG>;
    (void)batch;
    hipLaunchKernelGGL(k_proj_cols<LOGG>, dim3(a.units), dim3(C::WG), 0, st, a);
    return hipGetLastError();
}
template <int LOGM>
static hipError_t proj_polar_t(const ProjPolarArgs& a, int batch, hipStream_t st) {
    using C = ProjPolarCfg<LOGM>;
    const int pairs = (a.V + 1) / 2;
    hipLaunchKernelGGL(k_proj_polar<LOGM>, dim3((pairs + C::F - 1) / C::F, batch), dim3(C::WG), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_proj_rows(const bst_plan_s& p, const ProjRowArgs& a, int batch, hipStream_t st) {
    BST_SWITCH_LOG(p.logG, proj_rows_t, a, batch, st)
}
hipError_t launch_proj_cols(const bst_plan_s& p, const ProjColArgs& a, int batch, hipStream_t st) {
    BST_SWITCH_LOG(p.logG, proj_cols_t, a, batch, st)
}
hipError_t launch_proj_polar(const bst_plan_s& p, const ProjPolarArgs& a, int batch, hipStream_t st) {
    BST_SWITCH_LOG(p.logM, proj_polar_t, a, batch, st)
}
hipError_t launch_proj_gather(const bst_plan_s& p, const ProjGatherArgs& a, hipStream_t st) {
    (void)p;
    const int groups = (a.batch + kProjInterleave - 1) / kProjInterleave;
    const int angles = a.samples / a.half_m;
    const int tiles = ((a.half_m + kProjTileRadii - 1) / kProjTileRadii) *
                      ((angles + kProjTileAngles - 1) / kProjTileAngles);
    hipLaunchKernelGGL(k_proj_gather, dim3(tiles, groups), dim3(kProjGatherThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace bst

BST_CHECK_MODULE(project)
