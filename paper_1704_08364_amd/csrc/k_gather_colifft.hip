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
// With linear radial taps the polar spectra of Q = 2 consecutive slices are
// stored interleaved, sample by sample, in cache-line tiles of 2 angles x 4
// samples (PolarTiles): one tap of one point reads both slices' values of a
// sample as 16 contiguous bytes, and the four samples of a point's two angle
// rows mostly share one or two lines (simulated over the 2048 x 4096 gather
// points of N = 2048 with two columns per block: 7.9 distinct 128-byte lines
// per wave and slice, against 9.9 for interleaved rows and 16.4 for one
// slice per row). A block therefore gathers both slices of a group at once;
// their column transforms run one after the other, each gathered column
// waiting in its own LDS region. Cubic taps keep one slice per group in plain
// rows (Q = 1), and uneven batches too (their slices differ in V).
//
// Blocks have 1024 threads for transforms of 4096 points or more and 512
// below, where two blocks share a compute unit and one block's transforms
// overlap the other's polar reads (gather_threads).
//
// Each thread keeps the interpolation coordinates of its E points in
// three registers each and reuses them for every slice of its chunk. They
// are exact to FP32 rounding although radius and angle indices reach a few
// thousand:
//   radius index r = |(a,b)| P_r/P_c from an FP64 square root;
//   angle index: an FP32 atan2 picks the interval [theta_j0, theta_j0+1), then
//   the offset inside it is atan2(cross, dot) of the point direction against
//   (cos theta_j0, sin theta_j0) from an FP64 table (cross and dot in FP64,
//   the small angle in FP32), so the fraction f carries no cancellation.
// Per slice, the column is inverse-transformed along b, and only the N rows
// that survive the crop are written, to a grid laid out [N/8][GT][8]
// (complex, GT >= G/2 columns per tile row): the 8 rows of a tile and
// neighbouring columns form contiguous runs, and the row kernel reads each
// 8-row tile contiguously.
//
// Gather rules (bilinear in (r, q)):
//   b >= 0: theta = atan2(b, a), sample as stored; b < 0: theta + pi, conjugate
//   (y(t, theta + pi) = y(-t, theta)); the angle neighbour past theta_{V-1}
//   is theta_0 with the conjugation flipped; radial samples m >= M/2 are zero.
//   Origin (0,0): dc_scale * sum_j dt*Y_j[0] (mean for FBP, kappa/dk * mean
//   for plain B).
#include "bst_internal.h"
#include "bst_check.h"
#include "fft_lds.h"

namespace bst {

// Threads per block of the gather kernel (the columns per block follow from
// it): 1024 for transforms of 4096 points and more (two columns of 4096; two
// 512-thread blocks of one column each per compute unit measured 14 % slower,
// their footprints no longer shared), 512 below (two blocks per compute
// unit, one transforming while the other gathers: 7-21 % faster at G = 1024
// and 2048 than one 1024-thread block).
#ifndef BST_GATHER_THREADS
#define BST_GATHER_THREADS 0
#endif
constexpr int gather_threads(int G) { return BST_GATHER_THREADS ? BST_GATHER_THREADS : (G >= 4096 ? 1024 : 512); }

// waves per SIMD the register allocation must leave room for
#ifndef BST_GATHER_WAVES
#define BST_GATHER_WAVES 4
#endif

// Word 3 of a CDNA buffer resource for plain dword data (32-bit data format,
// no swizzle, raw offsets).
constexpr int kBufferWord3 = 0x00020000;

// One slice group's polar block as a buffer resource: loads take a 32-bit
// byte offset in one VGPR against a base held in SGPRs, and read 0 past the
// end. The block holds at most 16384 x 4101 x 32 bytes (< 2^32).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t polar_rsrc(const float2* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(base), 0, (int)bytes, kBufferWord3);
}

__device__ __forceinline__ float4 load16(__amdgpu_buffer_rsrc_t r, unsigned off) {
    const auto q = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return make_float4(__uint_as_float(q[0]), __uint_as_float(q[1]), __uint_as_float(q[2]), __uint_as_float(q[3]));
}

template <int LOGG, int QV = kPolarSlices, int CAPT = 0>
struct GatherCfg {
    static constexpr int G = 1 << LOGG;
    static constexpr int Q = QV;                         // slices per polar group
    static constexpr int E = 8;                          // points (values) per thread
    static constexpr int T = G / E;
    static constexpr int CAP = CAPT ? CAPT : gather_threads(G);
    static constexpr int WAVES = BST_GATHER_WAVES;       // per SIMD, for the registers
    static constexpr int MAXT = CAP > T ? CAP : T;
    static constexpr int FL = 16384 / G;                 // LDS: two regions of about 70 KB
    static constexpr int F1 = FL < G / 2 ? FL : G / 2;   // no more columns than exist
    static constexpr int F2 = MAXT / T;
    static constexpr int F = F1 < F2 ? F1 : F2;          // columns per block
    static constexpr int WG = F * T;
    // transform stride in LDS (float2; a power of two, the columns' lanes
    // interleaved and their positions told apart by region_xor)
    static constexpr int STRIDE = G;
    static constexpr int REGION = F * STRIDE;            // one slice's F transforms
    static constexpr int NREG = Q < 2 ? Q : 2;           // LDS regions (parked slices)
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

// Interpolation stencil of one Cartesian point, fixed for all slices:
//   o0      sample index (one unit is the Q slices' values of one sample,
//           8 Q bytes) of the first radial tap of angle j0; the taps of j1
//           are one polar row further, or, when j1 wraps to angle 0, (V-1)
//           rows back. In the tiled layout of two slices (PolarTiles) bit 29
//           says the second radial tap starts the next tile (m0 = 3 mod 4) and
//           bit 30 that j0 is odd (j1 in the next tile row). Bit 31 flips the conjugation of the j0 taps
//           (non-uniform angles, below theta_0, where the j0 neighbour is the
//           image theta_{V-1} - pi);
//   g       radial fraction, its sign bit set when j1 wraps;
//   w1      angular weight f of the j1 taps, negative when they are
//           conjugated. The j0 taps have weight 1 - f and are conjugated for
//           the lower half-plane b < 0 (known at compile time from the
//           point's slot in the thread), unless bit 31 of o0 flips it.
// Points outside the radial data (and the origin, which the DC rule sets
// afterwards) point at the zero slots that end rows 0 and 1, so every point
// runs the same branch-free code.
struct Stencil {
    unsigned o0;
    float g, w1;
};
constexpr unsigned kOffsetMask = 0x7FFFFFFFu;
constexpr unsigned kSampleMask = 0x1FFFFFFFu;  // o0 without its flag bits

// Angles of a slice: the plan's table, or (uneven batches, a count per
// slice) the slice's own table of j pi / V, else j pi / V formed with
// sincospi; V / pi in FP32.
struct AngleView {
    int V;
    float vpi_f;
    const double2* ang;  // (cos, sin) theta_j, or nullptr: uniform, from sincospi
    __device__ __forceinline__ double2 dir(int j) const {
        if (ang) return ang[j];
        double s, c;
        sincospi((double)j / (double)V, &s, &c);
        return make_double2(c, s);
    }
};

// conjugation of the j0 taps of point e: the lower half-plane, flipped by bit
// e of `flips` (bit 31 of the point's o0, collected once per block)
template <bool NU>
__device__ __forceinline__ bool lower_j0(unsigned flips, int e, bool lower) {
    if constexpr (NU) return lower != (((flips >> e) & 1u) != 0u);
    return lower;
}

// Stencil of Cartesian point (col, bs); bs signed. NU: non-uniform angles.
// TENT: a wide point of the tent rule (|bs| <= B_col) gets bit 31 of o0 and
// its patch slot in the low bits; its polar reads go to the zero slots.
template <bool TILED>
__device__ __forceinline__ unsigned sample_code(const GatherArgs& a, int j, int m) {
    if constexpr (TILED)
        return (unsigned)PolarTiles{2, a.V, a.S}.sample(j, m) | ((unsigned)((m & 3) == 3) << 29) |
               ((unsigned)(j & 1) << 30);
    else
        return (unsigned)(j * a.S + m);
}

template <bool NU, bool TENT, bool TILED>
__device__ __forceinline__ Stencil point_stencil(int col, int bs, const GatherArgs& a, const AngleView& av) {
    Stencil st;
    st.o0 = sample_code<TILED>(a, 0, a.zero_slot);
    st.g = st.w1 = 0.f;
    if (col == 0 && bs == 0) return st;
    if constexpr (TENT) {
        const int2 tc = a.tent_cols[col];
        if (bs >= -tc.y && bs <= tc.y) {
            st.o0 = (unsigned)(tc.x + bs + tc.y) | 0x80000000u;
            return st;
        }
    }
    const double r = sqrt((double)(col * col + bs * bs)) * a.rscale;
    if (r >= (double)a.zero_slot) return st;
    const double mf = floor(r);
    const int m0 = (int)mf;

    // direction of the point on [0, pi): (x, y) with y >= 0
    const bool lower = bs < 0;
    const int x = lower ? -col : col;
    const int y = lower ? -bs : bs;
    int j0;
    float f;
    bool flip0 = false;
    if constexpr (!NU) {
        const float th = atan2f((float)y, (float)x);
        j0 = (int)floorf(th * av.vpi_f);
        j0 = j0 < 0 ? 0 : (j0 >= av.V ? av.V - 1 : j0);
        const double2 cs = av.dir(j0);
        const double cross = (double)y * cs.x - (double)x * cs.y;
        const double dot = (double)x * cs.x + (double)y * cs.y;
        // the angle from theta_j0 is about pi / V or less: for |tan| < 0.01
        // atan t = t (1 - t^2 / 3) to far below FP32 rounding (the next
        // term is t^5 / 5), which spares the per-point atan2 of every slice
        // in uneven batches
        const float cr = (float)cross, dt = (float)dot;
        if (fabsf(cr) < 0.01f * dt) {
            const float t = cr / dt;
            f = t * fmaf(-t * t, 1.f / 3.f, 1.f) * av.vpi_f;
        } else {
            f = atan2f(cr, dt) * av.vpi_f;
        }
        if (f < 0.f) {
            if (j0 > 0) { j0 -= 1; f += 1.f; } else { f = 0.f; }
        } else if (f >= 1.f) {
            if (j0 < av.V - 1) { j0 += 1; f -= 1.f; } else { f = 1.f; }
        }
    } else {
        // theta_j <= theta exactly when the cross product e_j x u is >= 0 (both
        // directions in [0, pi)): binary search for the last such j
        auto at_or_before = [&](int jj) {
            const double2 e = a.ang[jj];
            return (double)y * e.x - (double)x * e.y >= 0.0;
        };
        double ex, ey;  // direction of the lower neighbour
        if (!at_or_before(0)) {
            j0 = a.V - 1;  // below theta_0: the image theta_{V-1} - pi, conjugated
            flip0 = true;
            ex = -a.ang[j0].x;
            ey = -a.ang[j0].y;
        } else {
            int lo = 0, hi = a.V;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (at_or_before(mid)) lo = mid; else hi = mid;
            }
            j0 = lo;
            ex = a.ang[j0].x;
            ey = a.ang[j0].y;
        }
        const double cross = (double)y * ex - (double)x * ey;
        const double dot = (double)x * ex + (double)y * ey;
        f = fminf(fmaxf(atan2f((float)cross, (float)dot) * a.inv_gap[j0], 0.f), 1.f);
    }
    // past theta_{V-1} the neighbour is theta_0 + pi: conjugated (both
    // neighbours of a point below theta_0 are already in place)
    const bool wrap = (j0 + 1 == av.V);
    const bool conj1 = lower != (wrap && !flip0);
    st.o0 = sample_code<TILED>(a, j0, m0) | ((unsigned)flip0 << 31);
    st.g = __uint_as_float(__float_as_uint((float)(r - mf)) | ((unsigned)wrap << 31));
    st.w1 = conj1 ? -f : f;
    return st;
}

// Grid stores are non-temporal: the row kernel reads them only after this
// kernel ends, and 2 GB of them per 64 slices would otherwise evict the polar
// lines the gather reuses.
__device__ __forceinline__ void store_streaming(float2* p, float2 v) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    const f2v t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<f2v*>(p));
}

// Keys cubic convolution (a = -1/2) over samples m0-1 .. m0+2 at fraction g:
// the Catmull-Rom weights.
__device__ __forceinline__ float2 keys4(float2 sm, float2 s0, float2 s1, float2 s2, float g) {
    const float g2 = g * g, g3 = g2 * g;
    const float wm = 0.5f * (-g3 + 2.f * g2 - g);
    const float w0 = 0.5f * (3.f * g3 - 5.f * g2 + 2.f);
    const float w1 = 0.5f * (-3.f * g3 + 4.f * g2 + g);
    const float w2 = 0.5f * (g3 - g2);
    return make_float2(fmaf(w2, s2.x, fmaf(w1, s1.x, fmaf(w0, s0.x, wm * sm.x))),
                       fmaf(w2, s2.y, fmaf(w1, s1.y, fmaf(w0, s0.y, wm * sm.y))));
}
// Angular (linear) combination of the two rows' radial values: weight
// 1 - |w1| for the j0 row, conjugated in the lower half-plane, and w1 (sign =
// conjugation) for the j1 row.
__device__ __forceinline__ float2 angular(float2 u0, float2 u1, float w1, bool lower) {
    const float a0 = 1.f - fabsf(w1);
    const float w0 = lower ? -a0 : a0;
    return make_float2(fmaf(fabsf(w1), u1.x, a0 * u0.x), fmaf(w1, u1.y, w0 * u0.y));
}

// One polar row's taps for the Q slices: linear taps read the samples m0,
// m0+1 (16 Q bytes), cubic taps m0-1 .. m0+2 (32 Q bytes); then their radial
// values.
template <int TAPS, int Q>
__device__ __forceinline__ void load_row(__amdgpu_buffer_rsrc_t P, unsigned off, float4 (&q)[TAPS * Q / 2]) {
#pragma unroll
    for (int i = 0; i < TAPS * Q / 2; ++i) q[i] = load16(P, off + 16u * i);
}
// value of slice k at tap t: complex number t Q + k of the row's run
template <int Q>
__device__ __forceinline__ float2 tap(const float4* q, int t, int k) {
    const int i = t * Q + k;
    const float4& h = q[i >> 1];
    return (i & 1) ? make_float2(h.z, h.w) : make_float2(h.x, h.y);
}
template <int TAPS, int Q>
__device__ __forceinline__ void radial_row(const float4 (&q)[TAPS * Q / 2], float g, float2 (&u)[Q]) {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        if constexpr (TAPS == 2) {
            const float2 x0 = tap<Q>(q, 0, k), x1 = tap<Q>(q, 1, k);
            u[k] = make_float2(fmaf(g, x1.x - x0.x, x0.x), fmaf(g, x1.y - x0.y, x0.y));
        } else {
            u[k] = keys4(tap<Q>(q, 0, k), tap<Q>(q, 1, k), tap<Q>(q, 2, k), tap<Q>(q, 3, k), g);
        }
    }
}

// Points of a thread whose reads are issued together. Every variant reads one
// point at a time: a point's four 16-byte reads mostly share one or two cache
// lines, and with fewer reads in flight the lines are still in L1 when the
// next point of a neighbouring lane needs them (two points at a time measured
// 2 % slower with the tiled layout, four 30 % slower, spilling; before the
// tiling, interleaved rows of two slices ran fastest with two).
#ifndef BST_GATHER_INFLIGHT
#define BST_GATHER_INFLIGHT 1
#endif
#ifndef BST_GATHER_INFLIGHT_OTHER
#define BST_GATHER_INFLIGHT_OTHER 1
#endif

// One block's work: columns lblock * F .. + F - 1 for the slices
// [s_begin, s_end) (whole groups of Q). The slices share one angle set: the
// plan's, or (per-slice counts) that of slice s_begin.
template <int LOGG, int TAPS, bool NU, bool TENT, int Q, int CAPT = 0>
__device__ __forceinline__ void gather_body(const GatherArgs& a, int lblock, int s_begin, int s_end) {
    using C = GatherCfg<LOGG, Q, CAPT>;
    constexpr int G = C::G, T = C::T, F = C::F, E = C::E;
    constexpr unsigned kSampleBytes = Q * sizeof(float2);
    constexpr bool TILED = Q == 2 && TAPS == 2;  // the 2 x 4 x 2 tiles of PolarTiles
    __shared__ float2 lds[C::NREG * C::REGION];  // one region per parked slice
    __shared__ float red[(C::WG + 63) / 64];
    const int fid = threadIdx.x % F;
    const int j = threadIdx.x / F;
    const int col = lblock * F + fid;
    const int V = a.Vs ? a.Vs[s_begin] : a.V;  // this chunk's projections
    const double2* ang = a.Vs ? (a.ang_off ? a.ang + a.ang_off[s_begin] : nullptr) : a.ang;
    const AngleView av{V, a.Vs ? (float)((double)V / M_PI) : a.vpi_f, ang};
    const float dc_scale = a.Vs ? a.dc_rule / (float)V : a.dc_scale;
    const bool live = col < G / 2;
    const FftTwiddles<LOGG, +1, E> tw(j, a.tw);

    // Stencils: computed in a rolled loop (one copy of the trigonometry in
    // registers), staged through the still unused transform LDS in chunks of
    // CH points, then held in registers for the whole chunk of slices.
    constexpr int CH = E == 8 ? 2 : 4;
    constexpr int NW = 3;  // words per stencil
    Stencil pt[E];
    static_assert(C::NREG * C::REGION * 2 >= C::WG * CH * NW, "stencil staging needs LDS");
    unsigned* stage = reinterpret_cast<unsigned*>(lds);
#pragma unroll
    for (int c0 = 0; c0 < E; c0 += CH) {
#pragma unroll 1
        for (int h = 0; h < CH; ++h) {
            const int b = j + (c0 + h) * T;
            const int bs = b < G / 2 ? b : b - G;
            const Stencil st = point_stencil<NU, TENT, TILED>(live ? col : 0, live ? bs : 0, a, av);
            unsigned* d = stage + (h * NW) * C::WG + threadIdx.x;
            d[0] = st.o0;
            d[C::WG] = __float_as_uint(st.g);
            d[2 * C::WG] = __float_as_uint(st.w1);
        }
#pragma unroll
        for (int h = 0; h < CH; ++h) {
            const unsigned* d = stage + (h * NW) * C::WG + threadIdx.x;
            pt[c0 + h].o0 = d[0];
            pt[c0 + h].g = __uint_as_float(d[C::WG]);
            pt[c0 + h].w1 = __uint_as_float(d[2 * C::WG]);
        }
    }
    __syncthreads();  // the transforms reuse this LDS
    // non-uniform angles: the j0 conjugation flips move to one bit mask; the
    // tent rule: wide points likewise (their o0 keeps the patch slot)
    unsigned flips = 0u, wide = 0u;
    if constexpr (NU || TENT) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            (NU ? flips : wide) |= (pt[e].o0 >> 31) << e;
            pt[e].o0 &= kOffsetMask;
        }
    }
    const unsigned zcode = sample_code<TILED>(a, 0, a.zero_slot);  // a zero sample
    const unsigned zoff = (zcode & kSampleMask) * kSampleBytes;

    const int half_n = a.N >> 1;
    const PolarTiles lay{Q, a.V, a.S};
    const unsigned group_bytes = (unsigned)(lay.group_elems() * sizeof(float2));
    const unsigned row_bytes = (unsigned)a.S * kSampleBytes;
    const unsigned wrap_bytes = 0u - (unsigned)(V - 1) * row_bytes;  // back to row 0
    // tiled: from angle j to j + 1 (j even: the tile's second half; j odd:
    // the next tile row's first), and from angle V - 1 back to angle 0
    const unsigned tile_row_bytes = (unsigned)lay.tiles_per_row() * 128u;
    const unsigned tile_next = tile_row_bytes - 64u;
    const unsigned tile_wrap = 0u - (unsigned)((V - 1) >> 1) * tile_row_bytes - (unsigned)((V - 1) & 1) * 64u;
    // column fid's LDS regions: slice 0 of a group at byte off0, slice 1 at off1
    const unsigned off0 = (unsigned)(fid * C::STRIDE) * 8u;
    const unsigned off1 = off0 + (unsigned)((C::NREG - 1) * C::REGION) * 8u;
    const int xm = region_xor<LOGG, F>(fid);
    for (int s0 = s_begin; s0 < s_end; s0 += Q) {
        const int nq = min(Q, s_end - s0);  // slices of this group in the batch
        // Re-derive the lane's row index each group: otherwise every address
        // that depends on it (LDS passes, grid stores) is hoisted out of the
        // loop and held in registers, which spills.
        int jv = j;
        asm volatile("" : "+v"(jv));
        const unsigned pj0 = lds_byte(off0, lds_swz<E>(jv), xm);  // the thread's first point
        const unsigned pj1 = lds_byte(off1, lds_swz<E>(jv), xm);
        const __amdgpu_buffer_rsrc_t P = polar_rsrc(a.polar + (size_t)(s0 / Q) * lay.group_elems(), group_bytes);
        float dcv[Q];
        if (lblock == 0) {
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                float acc = 0.f;
                if (k < nq)
                    for (int i = threadIdx.x; i < V; i += C::WG) acc += a.dc[(size_t)(s0 + k) * a.V + i];
                dcv[k] = block_sum<C::WG>(acc, red) * dc_scale;
            }
        }
        // gather: each slice of the group waits in its own LDS region
        constexpr int H = (TAPS == 2 && !NU && !TENT) ? BST_GATHER_INFLIGHT : BST_GATHER_INFLIGHT_OTHER;
        static_assert(E % H == 0, "whole groups of points");
#pragma unroll
        for (int h0 = 0; h0 < E; h0 += H) {
            float4 qa[H][TAPS * Q / 2], qb[H][TAPS * Q / 2];
#pragma unroll
            for (int i = 0; i < H; ++i) {
                const Stencil& st = pt[h0 + i];
                const bool wrap = __float_as_uint(st.g) >> 31;
                const bool zero = TENT && ((wide >> (h0 + i)) & 1u);
                if constexpr (TILED) {
                    // (j0, m0) and (j0, m0 + 1): 16 bytes apart, or 80 across a tile edge
                    const unsigned code = zero ? zcode : st.o0;
                    const unsigned oa = BST_IDX((code & kSampleMask) * 16u, group_bytes - 15u, 0);
                    const unsigned ob = BST_IDX(oa + (((code >> 29) & 1u) ? 80u : 16u), group_bytes - 15u, 0);
                    const unsigned d1 = wrap ? tile_wrap : (((code >> 30) & 1u) ? tile_next : 64u);
                    qa[i][0] = load16(P, oa);
                    qa[i][1] = load16(P, ob);
                    qb[i][0] = load16(P, BST_IDX(oa + d1, group_bytes - 15u, 0));
                    qb[i][1] = load16(P, BST_IDX(ob + d1, group_bytes - 15u, 0));
                } else {
                    constexpr unsigned kLast = TAPS * kSampleBytes - 1u;  // bytes read past the offset
                    const unsigned o0 = BST_IDX(zero ? zoff : st.o0 * kSampleBytes, group_bytes - kLast, 0);
                    const unsigned o1 = BST_IDX(o0 + (wrap ? wrap_bytes : row_bytes), group_bytes - kLast, 0);
                    load_row<TAPS, Q>(P, o0, qa[i]);
                    load_row<TAPS, Q>(P, o1, qb[i]);
                }
            }
#pragma unroll
            for (int i = 0; i < H; ++i) {
                const int e = h0 + i;
                const Stencil& st = pt[e];
                const float g = fabsf(st.g);
                float2 u0[Q], u1[Q], val[Q];
                radial_row<TAPS, Q>(qa[i], g, u0);
                radial_row<TAPS, Q>(qb[i], g, u1);
#pragma unroll
                for (int k = 0; k < Q; ++k) val[k] = angular(u0[k], u1[k], st.w1, lower_j0<NU>(flips, e, 2 * e >= E));
                if constexpr (TENT) {
                    // wide points: the value pre-gathered over their tent of angles
                    if ((wide >> e) & 1u) {
#pragma unroll
                        for (int k = 0; k < Q; ++k) {
                            const int sk = min(s0 + k, a.batch - 1);
                            val[k] = a.patch[(size_t)sk * a.tent_w + BST_IDX(st.o0, (unsigned)a.tent_w, 1)];
                        }
                    }
                }
                // origin: column 0, row 0 is thread j = 0's first point
                if (e == 0 && col == 0 && jv == 0) {
#pragma unroll
                    for (int k = 0; k < Q; ++k) val[k] = make_float2(dcv[k], 0.f);
                }
                lds_at(lds, pj0 ^ swz_bytes<E>(e * T)) = val[0];
                if constexpr (Q > 1) lds_at(lds, pj1 ^ swz_bytes<E>(e * T)) = val[1];
            }
            asm volatile("" ::: "memory");
        }
        __syncthreads();

        // One transform per iteration, the loop kept rolled: unrolled, the
        // transforms share address arithmetic that then stays live across
        // all of them and spills. Each slice comes from its LDS region.
#pragma unroll 1
        for (int k = 0; k < nq; ++k) {
            int jk = jv;
            asm volatile("" : "+v"(jk));
            const unsigned offk = (k & 1) ? off1 : off0;
            const unsigned pk = lds_byte(offk, lds_swz<E>(jk), xm);
            float2 v[E];
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = lds_at(lds, pk ^ swz_bytes<E>(e * T));
            __syncthreads();  // every lane has its inputs before the first pass writes
            FftTwiddles<LOGG, +1, E> twl = tw;
            twl.pin();
            fft<LOGG, +1, E>(v, lds, offk, jk, twl, xm);
            if (live) {
                float2* D = a.grid + (size_t)(s0 + k) * a.N * a.GT;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int y = jk + e * T;
                    const int p = (y + half_n) & (G - 1);
                    if (p < a.N)
                        store_streaming(&D[BST_IDX(((size_t)(p >> 3) * a.GT + col) * 8 + (p & 7),
                                                   (size_t)a.N * a.GT, 2)], v[e]);
                }
            }
        }
    }
}

template <int LOGG, int TAPS, bool NU, bool TENT>
__global__ void __launch_bounds__((GatherCfg<LOGG, polar_group(TAPS)>::WG))
__attribute__((amdgpu_waves_per_eu(GatherCfg<LOGG, polar_group(TAPS)>::WAVES, 8))) k_gather_colifft(GatherArgs a) {
    const int s_begin = blockIdx.y * a.slices_per_block;  // a multiple of Q
    gather_body<LOGG, TAPS, NU, TENT, polar_group(TAPS)>(a, xcd_contiguous(blockIdx.x, gridDim.x), s_begin,
                                                         min(a.batch, s_begin + a.slices_per_block));
}

// Persistent launch of uneven batches (one slice per group, uniform angles):
// every block walks the work list (slice, column block) in steps of the grid,
// the blocks of one XCD taking contiguous items (the neighbouring columns of
// one slice, which read the same polar lines). Blocks of 1024 threads at
// every length: the classes' persistent kernels run side by side, and
// 512-thread blocks measured slower there.
constexpr int kItemsThreads = 1024;
template <int LOGG, int TAPS>
__global__ void __launch_bounds__((GatherCfg<LOGG, 1, kItemsThreads>::WG))
__attribute__((amdgpu_waves_per_eu(GatherCfg<LOGG, 1, kItemsThreads>::WAVES, 8))) k_gather_items(GatherArgs a) {
    const int local = xcd_contiguous(blockIdx.x, gridDim.x);
    for (int base = 0; base < a.n_items; base += gridDim.x) {
        const int it = base + local;
        if (it >= a.n_items) break;
        const int2 w = a.items[it];
        __syncthreads();  // the previous item's LDS reads are done
        gather_body<LOGG, TAPS, false, false, 1, kItemsThreads>(a, w.y, w.x, w.x + 1);
    }
}

template <int LOGG, int TAPS>
static hipError_t launch_gather_t(const GatherArgs& a, hipStream_t st) {
    using C = GatherCfg<LOGG, polar_group(TAPS)>;
    const int cols = C::G / 2;
    if (a.slices_per_block <= 0 || a.slices_per_block % C::Q != 0) return hipErrorInvalidValue;
    const int chunks = (a.batch + a.slices_per_block - 1) / a.slices_per_block;
    dim3 grid((cols + C::F - 1) / C::F, chunks);
    if (a.tent_cols) {
        // tent rule: uniform angles and linear radial taps only (checked by the plan)
        if constexpr (TAPS == 2)
            hipLaunchKernelGGL((k_gather_colifft<LOGG, TAPS, false, true>), grid, dim3(C::WG), 0, st, a);
        else
            return hipErrorInvalidValue;
    } else if (a.uniform) {
        hipLaunchKernelGGL((k_gather_colifft<LOGG, TAPS, false, false>), grid, dim3(C::WG), 0, st, a);
    } else {
        hipLaunchKernelGGL((k_gather_colifft<LOGG, TAPS, true, false>), grid, dim3(C::WG), 0, st, a);
    }
    return hipGetLastError();
}

static_assert(kTentSlices % kPolarSlices == 0, "a tent group spans whole polar groups");

// Tent rule, step 1: the first `rows` radial samples of every angle,
// radius-major with kTentSlices slices interleaved ([group][m][j][slice]), so
// one angular tap of step 2 reads its slices' values as one contiguous 64-byte
// run. A block moves a tile of 32 radii x 8 angles of every slice of its
// group through LDS: reads are 32-sample runs of a polar row, writes are the
// tile's 8 angles x 8 slices of each radius, one contiguous 512-byte run.
// Slices past the batch are written as zeros.
__global__ void __launch_bounds__(256) k_tent_transpose(TentArgs a, int batch) {
    __shared__ float2 tile[kTentSlices][8][33];
    const int grp = blockIdx.z;
    const int m0 = blockIdx.x * 32, j0 = blockIdx.y * 8;
    // reads follow the interleaved polar layout: the Q slices of one sample,
    // then consecutive samples (runs of 4 samples with Q = 2, 32 otherwise)
    constexpr int Q = kPolarSlices, NG = kTentSlices / kPolarSlices;
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int idx = it * 256 + threadIdx.x;
        const int k4 = idx % Q, m = (idx / Q) & 31, kh = (idx / (32 * Q)) % NG, j = idx / 256;
        const int k = kh * Q + k4;
        const int s = grp * kTentSlices + k;
        float2 v = make_float2(0.f, 0.f);
        if (s < batch && j0 + j < a.V && m0 + m < a.rows) {
            const PolarTiles lay{Q, a.V, a.S};
            v = a.polar[(size_t)(s / Q) * lay.group_elems() +
                        lay.sample(j0 + j, BST_IDX(a.lead + m0 + m, a.S, 3)) * Q + k4];
        }
        tile[k][j][m] = v;
    }
    __syncthreads();
    float2* Tg = a.trans + (size_t)grp * a.rows * a.V * kTentSlices;
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int idx = it * 256 + threadIdx.x;
        const int k = idx & 7, j = (idx >> 3) & 7, m = idx >> 6;
        if (m0 + m < a.rows && j0 + j < a.V)
            Tg[BST_IDX(((size_t)(m0 + m) * a.V + j0 + j) * kTentSlices + k, (size_t)a.rows * a.V * kTentSlices, 4)] =
                tile[k][j][m];
    }
}

// Tent rule, step 2: one thread per chunk of at most kTentChunk angle taps
// of one wide point, for kTentSlices slices. The point (a, b) of the chunk's
// slot comes from the column table; its taps are the angle indices j of the
// period-pi continuation with |q - j| < h, weights (1 - |q - j| / h), on the
// two radial samples m0, m0 + 1 (linear weights); j outside [0, V) reads the
// conjugated image of j mod V, and the lower half-plane conjugates the
// result. Coordinates are formed in FP64 as on the host. Splitting the long
// tap ranges near the origin (over a thousand taps) into chunks keeps every
// thread's loop short.
__device__ __forceinline__ int tent_column(const TentArgs& a, int slot) {
    // the last column whose first slot is <= slot
    int lo = 0, hi = a.ncols - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.cols[mid].x <= slot) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(256) k_tent_chunks(TentArgs a, int batch) {
    // neighbouring chunks read the same angle taps: keep them on one XCD
    const int c = xcd_contiguous(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const int s0 = blockIdx.y * kTentSlices;
    if (c >= a.C) return;
    const int ns = min(kTentSlices, batch - s0);
    const int4 ch = a.chunk[c];
    const int col = BST_IDX(tent_column(a, ch.x), a.ncols, 5);
    const int2 tc = a.cols[col];
    const int b = ch.x - tc.x - tc.y;
    const double rho = sqrt((double)col * col + (double)b * b);
    const double phi = atan2((double)b, (double)col);
    const bool lower = phi < 0.0;
    const double q = (lower ? phi + M_PI : phi) * ((double)a.V / M_PI);
    const double h = (double)a.V / (M_PI * rho);
    const double r = rho * a.rscale;
    const int m0 = BST_IDX((int)floor(r), a.rows, 6);
    const float g = (float)(r - (double)m0);
    const float w1r = m0 + 1 < a.rows ? g : 0.f;  // samples past M/2 are zero
    const float inv_h = (float)(1.0 / h);
    // the slice group's radius-major rows m0 and m0 + 1, 8 slices per angle
    const float4* T0 = reinterpret_cast<const float4*>(
        a.trans + ((size_t)blockIdx.y * a.rows + m0) * a.V * kTentSlices);
    const float4* T1 = T0 + (m0 + 1 < a.rows ? (size_t)a.V * (kTentSlices / 2) : 0);
    float ax[kTentSlices], ay[kTentSlices];
#pragma unroll
    for (int k = 0; k < kTentSlices; ++k) ax[k] = ay[k] = 0.f;
    float total = 0.f;
    for (int jc = ch.y; jc <= ch.z; ++jc) {
        const float w = 1.f - fabsf((float)(q - (double)jc)) * inv_h;
        if (w <= 0.f) continue;
        total += w;
        const bool flip = jc < 0 || jc >= a.V;
        const int jj = BST_IDX(jc < 0 ? jc + a.V : (jc >= a.V ? jc - a.V : jc), a.V, 7);
        const float wy = flip ? -w : w;
        float2 v0[kTentSlices], v1[kTentSlices];
#pragma unroll
        for (int k = 0; k < kTentSlices; k += 2) {
            const float4 p0 = T0[(size_t)jj * (kTentSlices / 2) + k / 2];
            const float4 p1 = T1[(size_t)jj * (kTentSlices / 2) + k / 2];
            v0[k] = make_float2(p0.x, p0.y);
            v0[k + 1] = make_float2(p0.z, p0.w);
            v1[k] = make_float2(p1.x, p1.y);
            v1[k + 1] = make_float2(p1.z, p1.w);
        }
#pragma unroll
        for (int k = 0; k < kTentSlices; ++k) {
            const float vx = fmaf(w1r, v1[k].x - v0[k].x, v0[k].x);
            const float vy = fmaf(w1r, v1[k].y - v0[k].y, v0[k].y);
            ax[k] = fmaf(w, vx, ax[k]);
            ay[k] = fmaf(wy, vy, ay[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < kTentSlices; ++k)
        if (k < ns) a.part[(size_t)(s0 + k) * a.C + c] = make_float2(ax[k], lower ? -ay[k] : ay[k]);
    if (blockIdx.y == 0) a.wsum[c] = total;
}

// Tent rule, step 3: each wide point's value is the sum of its chunks'
// partial sums over the sum of their weights (chunks in order).
__global__ void __launch_bounds__(256) k_tent_reduce(TentArgs a) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= a.W) return;
    const int c1 = a.coff[i + 1];
    float ax = 0.f, ay = 0.f, tot = 0.f;
    for (int c = a.coff[i]; c < c1; ++c) {
        const float2 p = a.part[(size_t)s * a.C + c];
        ax += p.x;
        ay += p.y;
        tot += a.wsum[c];
    }
    const float inv = tot > 0.f ? 1.f / tot : 0.f;
    a.patch[(size_t)s * a.W + i] = make_float2(ax * inv, ay * inv);
}

hipError_t launch_tent(const bst_plan_s& p, const TentArgs& a, int batch, hipStream_t st) {
    (void)p;
    if (a.W <= 0) return hipSuccess;
    const int groups = (batch + kTentSlices - 1) / kTentSlices;
    hipLaunchKernelGGL(k_tent_transpose, dim3((a.rows + 31) / 32, (a.V + 7) / 8, groups), dim3(256), 0, st, a,
                       batch);
    if (a.C > 0)
        hipLaunchKernelGGL(k_tent_chunks, dim3((a.C + 255) / 256, (batch + kTentSlices - 1) / kTentSlices), dim3(256),
                           0, st, a, batch);
    hipLaunchKernelGGL(k_tent_reduce, dim3((a.W + 255) / 256, batch), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int LOGG>
static hipError_t launch_gather_items_t(const GatherArgs& a, int taps, int blocks, hipStream_t st) {
    using C = GatherCfg<LOGG, 1, kItemsThreads>;
    if (taps == 4) hipLaunchKernelGGL((k_gather_items<LOGG, 4>), dim3(blocks), dim3(C::WG), 0, st, a);
    else hipLaunchKernelGGL((k_gather_items<LOGG, 2>), dim3(blocks), dim3(C::WG), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gather_items(const bst_plan_s& p, const GatherArgs& a, int blocks, hipStream_t st) {
    if (a.tent_cols || !a.Vs) return hipErrorInvalidValue;
    switch (p.logG) {
        case 4: return launch_gather_items_t<4>(a, p.taps, blocks, st);
        case 5: return launch_gather_items_t<5>(a, p.taps, blocks, st);
        case 6: return launch_gather_items_t<6>(a, p.taps, blocks, st);
        case 7: return launch_gather_items_t<7>(a, p.taps, blocks, st);
        case 8: return launch_gather_items_t<8>(a, p.taps, blocks, st);
        case 9: return launch_gather_items_t<9>(a, p.taps, blocks, st);
        case 10: return launch_gather_items_t<10>(a, p.taps, blocks, st);
        case 11: return launch_gather_items_t<11>(a, p.taps, blocks, st);
        case 12: return launch_gather_items_t<12>(a, p.taps, blocks, st);
        case 13: return launch_gather_items_t<13>(a, p.taps, blocks, st);
        default: return hipErrorInvalidValue;
    }
}

template <int LOGG>
static int gather_cols_t() {
    using C = GatherCfg<LOGG, 1, kItemsThreads>;
    return (C::G / 2 + C::F - 1) / C::F;
}

int gather_blocks_per_slice(const bst_plan_s& p) {
    switch (p.logG) {
        case 4: return gather_cols_t<4>();
        case 5: return gather_cols_t<5>();
        case 6: return gather_cols_t<6>();
        case 7: return gather_cols_t<7>();
        case 8: return gather_cols_t<8>();
        case 9: return gather_cols_t<9>();
        case 10: return gather_cols_t<10>();
        case 11: return gather_cols_t<11>();
        case 12: return gather_cols_t<12>();
        case 13: return gather_cols_t<13>();
        default: return 0;
    }
}

hipError_t launch_gather_colifft(const bst_plan_s& p, const GatherArgs& a, hipStream_t st) {
    const bool cubic = p.taps == 4;
    switch (p.logG) {
        case 4: return cubic ? launch_gather_t<4, 4>(a, st) : launch_gather_t<4, 2>(a, st);
        case 5: return cubic ? launch_gather_t<5, 4>(a, st) : launch_gather_t<5, 2>(a, st);
        case 6: return cubic ? launch_gather_t<6, 4>(a, st) : launch_gather_t<6, 2>(a, st);
        case 7: return cubic ? launch_gather_t<7, 4>(a, st) : launch_gather_t<7, 2>(a, st);
        case 8: return cubic ? launch_gather_t<8, 4>(a, st) : launch_gather_t<8, 2>(a, st);
        case 9: return cubic ? launch_gather_t<9, 4>(a, st) : launch_gather_t<9, 2>(a, st);
        case 10: return cubic ? launch_gather_t<10, 4>(a, st) : launch_gather_t<10, 2>(a, st);
        case 11: return cubic ? launch_gather_t<11, 4>(a, st) : launch_gather_t<11, 2>(a, st);
        case 12: return cubic ? launch_gather_t<12, 4>(a, st) : launch_gather_t<12, 2>(a, st);
        case 13: return cubic ? launch_gather_t<13, 4>(a, st) : launch_gather_t<13, 2>(a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bst

BST_CHECK_MODULE(gather)
