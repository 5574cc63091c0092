// k_spectrum.hip -- steps P0-P4 of the BST (Section 2): taper, zero pad,
// 1D FFT along the detector axis and the radial weight, fused in one kernel.
//
// Two projections j, j+1 of a slice share one complex FFT of length M:
// z = w.y_j + i w.y_{j+1}, placed so that t = 0 sits at index 0
// (z[(i - n/2) mod M] = w[i] y[i]); the padded zeros exist only in registers.
// After the transform Z, the two real spectra separate as
//   Y_j[m] = (Z[m] + conj Z[M-m]) / 2,   Y_{j+1}[m] = (Z[m] - conj Z[M-m]) / (2i),
// and each is multiplied by the complex weight dt*K[m]*A(sigma_m)*exp(2 pi i
// sigma_m beta dt) (K = 1/sigma for plain B, 1 for FBP, 0 at m = M/2; A the
// apodising window; beta a known rotation-axis offset). With raw counts the
// load forms y = -log((I - D)/(I0 - D)) first (flat/dark normalisation).
// The polar spectra of a group of Q consecutive slices are stored interleaved
// (sample m of projection j of the group's slices in 8 Q contiguous bytes),
// because the gather reads all of them at every tap; groups of two slices in
// cache-line tiles of neighbouring angles and samples (PolarTiles).
// Output rows hold m = 0..M/2-1 followed by zero slots, so the gather may read
// past the last sample without a bound test: two for linear radial
// interpolation (samples m0, m0+1), four plus a leading conj Yh[1] (the
// sample at m = -1) for cubic interpolation (samples m0-1 .. m0+2).
// The unweighted DC values dt*Y_j[0] go to a separate array for the origin rule.
// With monopole subtraction (plain B), a reduction kernel first sums each
// slice's sinogram (partial sums of kMassChunks blocks); the spectrum kernel
// turns them into the mass m and loads y[i] - m phi[i] in place of y[i].
#include "bst_internal.h"
#include "fft_lds.h"
#include "bst_check.h"
#include "monopole.h"

// waves per SIMD the register allocation must leave room for
#ifndef BST_SPEC_WAVES
#define BST_SPEC_WAVES 4
#endif
// projection pairs per block in turn (the next pair's detector data read
// while the current one is transformed): one, since with conflict-free LDS
// exchanges more resident blocks hide the reads better than the prefetch
// (64 x 2048^2: 0.67 ms with two pairs per block, 0.62 ms with one)
#ifndef BST_SPEC_PAIRS
#define BST_SPEC_PAIRS 1
#endif

namespace bst {

// Projection pairs per block in turn: the prefetch needs registers for one
// more pair's data slots, which only the P_r >= 2 plain-input variants have
// to spare.
template <int LOGP, bool COUNTS, bool MONO>
constexpr int spec_pairs() { return (LOGP >= 1 && !COUNTS && !MONO) ? BST_SPEC_PAIRS : 1; }

// Partial sums of each slice's sinogram for the monopole mass: block (c, s)
// adds up lines j = c, c + kMassChunks, ... (raw counts normalised as the
// spectrum kernel does), every thread over a fixed set of elements and the
// block in a fixed tree, so each call gives the same sums.
constexpr int kMassThreads = 256;

template <bool COUNTS>
__global__ void __launch_bounds__(kMassThreads) k_mass(MassArgs a) {
    __shared__ float red[kMassThreads / 64];
    const int c = blockIdx.x, s = blockIdx.y;
    const float* base = a.sino_list ? a.sino_list[s] : a.sino + (size_t)s * a.V * a.n;
    const int V = a.Vs ? a.Vs[s] : a.V;
    const int lines = c < V ? (V - 1 - c) / kMassChunks + 1 : 0;
    const int logn = __ffs(a.n) - 1;  // n is a power of two
    const long long items = (long long)lines << logn;
    const float* fs = COUNTS ? a.flat + (size_t)s * a.n : nullptr;
    const float* ds = COUNTS ? a.dark + (size_t)s * a.n : nullptr;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (long long it0 = threadIdx.x; it0 < items; it0 += 4LL * kMassThreads) {
        float x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long long it = it0 + (long long)u * kMassThreads;
            const bool ok = it < items;
            const long long itc = ok ? it : 0;
            const int l = (int)(itc >> logn);
            const int i = (int)(itc & (a.n - 1));
            float v = base[BST_IDX((size_t)(c + l * kMassChunks) * a.n + i, (size_t)V * a.n, 0)];
            if constexpr (COUNTS) {
                const float inv = 1.0f / (fs[i] - ds[i]);
                v = -logf((v - ds[i]) * inv);
            }
            x[u] = ok ? v : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += x[u];
    }
    float v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
#pragma unroll
        for (int w = 0; w < kMassThreads / 64; ++w) t += red[w];
        a.part[(size_t)s * kMassChunks + c] = t;
    }
}

template <int LOGM, int Q>
struct SpecCfg {
    static constexpr int M = 1 << LOGM;
    static constexpr int T = M / 16;                     // threads per transform
    static constexpr int TP = Q * T;                     // per projection pair: one transform per slice
    // projection pairs per block: blocks of at least 256 threads (one-slice
    // groups at M = 4096: 0.665 ms in 512-thread blocks, 0.641 ms in 256)
    static constexpr int FP = TP >= 256 ? 1 : 256 / TP;
    static constexpr int WG = FP * TP;
    static constexpr int MV = (M / 2) / TP;              // output samples per thread and pair
};

// LOGP = log2(P_r). Thread j's padded positions k = j + e*T hold data only for
// e < E0 or e >= 16 - E0 (E0 = 8 / P_r): the middle of every line is padding,
// known at compile time, so it is never loaded. COUNTS: the input is raw
// counts with per-slice flat and dark fields.
// Unpadded raw counts with the monopole hold the most per-thread state: they
// get room for 3 waves per SIMD instead of spilling.
template <int LOGP, bool COUNTS, bool MONO>
constexpr int spec_waves() { return (MONO && COUNTS && LOGP == 0) ? 3 : BST_SPEC_WAVES; }

// One block: FP projection pairs (PAIRS of them in turn) of one group of
// kPolarSlices slices, one complex transform per slice and pair (so every
// slice's result is independent of the other slices). The epilogue separates
// the two real spectra of every transform and writes, for every sample m of
// each of the two projections, the group's slices' values side by side
// (8 Q contiguous bytes), so the polar rows come out interleaved as the
// gather reads them: sample PolarTiles{Q, V, S}.sample(j, lead + m) of group g.
// Slices of the last group past the batch read zeros.
// MONO: monopole subtraction, y[i] - m phi[i] (m from the partial sums).
// Q: slices per polar group (kPolarSlices for ordinary batches with linear
// taps, 1 with cubic taps and in the persistent launches of uneven batches).
// Block (bx, g): pair blocks bx of group g.
template <int LOGM, int LOGP, bool COUNTS, bool MONO, int Q>
__device__ __forceinline__ void spectrum_body(const SpecArgs& a, int batch, int bx, int g) {
    using C = SpecCfg<LOGM, Q>;
    constexpr int M = C::M, T = C::T, TP = C::TP;
    constexpr int E0 = 8 >> LOGP;
    constexpr int NQ = 2 * E0;  // data slots per thread
    __shared__ float2 lds[Q * C::FP * M];
    const int u = threadIdx.x / T;        // transform: pair u / Q, slice u % Q
    const int j = threadIdx.x - u * T;
    const int pl = u / Q, k = u % Q;
    const unsigned my_off = (unsigned)(u * M) * 8u;  // this transform's LDS region
    const int my_xm = contiguous_xor<LOGM, T>(u);
    const int s = g * Q + k;
    const bool vs = s < batch;
    const int h = a.n >> 1;
    constexpr int PAIRS = spec_pairs<LOGP, COUNTS, MONO>();
    const int npairs = (a.V + 1) >> 1;  // pairs of the layout's rows

    // detector bin of data slot q: positions e = q (q < E0) and e = 16 - 2*E0 + q (q >= E0)
    auto bin_of = [&](int q) {
        const int e = q < E0 ? q : 16 - 2 * E0 + q;
        const int kk = j + e * T;
        return kk < h ? kk + h : kk - M + h;
    };
    const int sc = vs ? s : 0;  // a slice past the batch reads slice 0, dropped below
    const float* base = a.sino_list ? a.sino_list[sc] : a.sino + (size_t)sc * a.V * a.n;
    const int Vk = a.Vs ? a.Vs[sc] : a.V;  // this slice's projections

    // Every global read of the thread is issued up front with no branch in
    // between: the data slots of both lines of the first pair (a missing
    // line -- an odd V, or a pair past the end -- reads line 0 and is
    // dropped by a select), the taper, flat and dark, the epilogue weights and
    // the twiddle anchors; these last are the same for every pair.
    auto load_lines = [&](int pair, float (&ra)[NQ], float (&rb)[NQ]) {
        const int ja = 2 * pair, jb = 2 * pair + 1;
        const float* ya = base + (size_t)(ja < Vk ? ja : 0) * a.n;
        const float* yb = base + (size_t)(jb < Vk ? jb : 0) * a.n;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int i = BST_IDX(bin_of(q), a.n, 1);
            ra[q] = ya[i];
            rb[q] = yb[i];
        }
    };
    float ra[NQ], rb[NQ], w[NQ];
    const int pair0 = bx * PAIRS * C::FP + pl;
    load_lines(pair0 < npairs ? pair0 : 0, ra, rb);
#pragma unroll
    for (int q = 0; q < NQ; ++q) w[q] = a.taper[bin_of(q)];
    float dk[COUNTS ? NQ : 1], fl[COUNTS ? NQ : 1];
    if constexpr (COUNTS) {
        const float* fs = a.flat + (size_t)sc * a.n;
        const float* ds = a.dark + (size_t)sc * a.n;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int i = bin_of(q);
            fl[q] = fs[i];
            dk[q] = ds[i];
        }
    }
    float mph[MONO ? NQ : 1];  // m phi at the thread's bins
    if constexpr (MONO) {
        const float m = monopole_mass(a.mono_part, sc, a.Vs ? a.mono_inv * (float)a.V / (float)Vk : a.mono_inv);
#pragma unroll
        for (int q = 0; q < NQ; ++q) mph[q] = m * a.mono_phi[bin_of(q)];
    }
    // epilogue: thread q of its pair handles samples m = q + i*TP
    const int qp = threadIdx.x - pl * TP;
    float2 kc[C::MV];
#pragma unroll
    for (int i = 0; i < C::MV; ++i) kc[i] = a.kc[qp + i * TP];
    const FftTwiddles<LOGM, -1, 16> tw(j, a.tw);

#pragma unroll
    for (int it = 0; it < PAIRS; ++it) {
        const int pair = pair0 + it * C::FP;
        const int ja = 2 * pair, jb = 2 * pair + 1;
        const bool va = ja < Vk && vs, vb = jb < Vk && vs;
        float na[NQ], nb[NQ];
        if (it + 1 < PAIRS) {
            const int nx = pair + C::FP;
            load_lines(nx < npairs ? nx : 0, na, nb);
        }

        float2 v[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = make_float2(0.f, 0.f);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            float xa = ra[q], xb = rb[q];
            if constexpr (COUNTS) {
                // flat/dark normalisation, y = -log((I - D) / (I0 - D))
                const float inv = 1.0f / (fl[q] - dk[q]);
                xa = -logf((xa - dk[q]) * inv);
                xb = -logf((xb - dk[q]) * inv);
            }
            if constexpr (MONO) {
                xa -= mph[q];
                xb -= mph[q];
            }
            v[q < E0 ? q : 16 - 2 * E0 + q] = make_float2(va ? w[q] * xa : 0.f, vb ? w[q] * xb : 0.f);
        }

        // fresh copies per pair, so that nothing derived from them is
        // computed once and held across the transforms (that spills)
        FftTwiddles<LOGM, -1, 16> twl = tw;
        twl.pin();
        int jv = j;
        asm volatile("" : "+v"(jv));
        fft<LOGM, -1>(v, lds, my_off, jv, twl, my_xm);

        const unsigned pj = lds_byte(my_off, lds_swz<16>(jv), my_xm);
#pragma unroll
        for (int e = 0; e < 16; ++e) lds_at(lds, pj ^ swz_bytes<16>(e * T)) = v[e];
        if (jv == 0) {
            if (va) a.dc[(size_t)s * a.V + BST_IDX(ja, a.V, 3)] = a.dt * v[0].x;
            if (vb) a.dc[(size_t)s * a.V + BST_IDX(jb, a.V, 3)] = a.dt * v[0].y;
        }
        __syncthreads();

        // separate the two real spectra of every slice's transform and store
        // rows ja and jb with the group's slices interleaved
        const bool wa = ja < a.V, wb = jb < a.V;

        const PolarTiles lay{Q, a.V, a.S};
        float2* grp = a.polar + (size_t)g * lay.group_elems();
        const int rja = wa ? ja : 0, rjb = wb ? jb : 0;
        // one sample of the Q slices: 8 Q bytes, as float2 (Q = 1) or float4 parts
        auto put = [&](int row, int slot, const float2 (&y)[Q], bool conj) {
            const float c = conj ? -1.f : 1.f;
            float2* at = grp + BST_IDX(lay.sample(row, slot), lay.group_elems() / Q, 2) * Q;
            if constexpr (Q == 1) {
                *at = make_float2(y[0].x, c * y[0].y);
            } else {
                float4* r4 = reinterpret_cast<float4*>(at);
#pragma unroll
                for (int t = 0; t < Q / 2; ++t)
                    r4[t] = make_float4(y[2 * t].x, c * y[2 * t].y, y[2 * t + 1].x, c * y[2 * t + 1].y);
            }
        };
        int qv = qp;
        asm volatile("" : "+v"(qv));
#pragma unroll
        for (int i = 0; i < C::MV; ++i) {
            const int m = qv + i * TP;  // 0 .. M/2-1
            const int mc = (M - m) & (M - 1);
            const int slot = BST_IDX(a.lead + m, a.S, 2);
            float2 ya[Q], yb[Q];
#pragma unroll
            for (int d = 0; d < Q; ++d) {
                // slice d's transform of this pair
                const unsigned zoff = (unsigned)((Q * pl + d) * M) * 8u;
                const int zxm = contiguous_xor<LOGM, T>(Q * pl + d);
                const float2 z = lds_at(lds, lds_byte(zoff, lds_swz<16>(m), zxm));
                const float2 zc = lds_at(lds, lds_byte(zoff, lds_swz<16>(mc), zxm));
                ya[d] = cmul(make_float2(0.5f * (z.x + zc.x), 0.5f * (z.y - zc.y)), kc[i]);
                yb[d] = cmul(make_float2(0.5f * (z.y + zc.y), -0.5f * (z.x - zc.x)), kc[i]);
            }
            if (wa) {
                put(rja, slot, ya, false);
                // the sample before 0 (cubic radial taps): Yh(-sigma) = conj Yh(sigma)
                if (a.lead && m == 1) put(rja, 0, ya, true);
            }
            if (wb) {
                put(rjb, slot, yb, false);
                if (a.lead && m == 1) put(rjb, 0, yb, true);
            }
        }
        for (int z = qv; z < a.tail; z += TP) {
            const int slot = BST_IDX(a.lead + M / 2 + z, a.S, 2);
            float2 zero[Q];
#pragma unroll
            for (int d = 0; d < Q; ++d) zero[d] = make_float2(0.f, 0.f);
            if (wa) put(rja, slot, zero, false);
            if (wb) put(rjb, slot, zero, false);
        }
        if (it + 1 < PAIRS) {
            __syncthreads();  // the next transforms overwrite this LDS
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                ra[q] = na[q];
                rb[q] = nb[q];
            }
        }
    }
}

template <int LOGM, int LOGP, bool COUNTS, bool MONO, int Q>
__global__ void __launch_bounds__((SpecCfg<LOGM, Q>::WG))
__attribute__((amdgpu_waves_per_eu(spec_waves<LOGP, COUNTS, MONO>(), 8))) k_spectrum(SpecArgs a, int batch) {
    spectrum_body<LOGM, LOGP, COUNTS, MONO, Q>(a, batch, blockIdx.x, blockIdx.y);
}

// Persistent launch: every block walks the work list (group, pair block) in
// steps of the grid, blocks of one XCD taking contiguous items.
template <int LOGM, int LOGP, bool COUNTS, bool MONO>
__global__ void __launch_bounds__((SpecCfg<LOGM, 1>::WG))
__attribute__((amdgpu_waves_per_eu(spec_waves<LOGP, COUNTS, MONO>(), 8))) k_spectrum_items(SpecArgs a, int batch) {
    const int local = xcd_contiguous(blockIdx.x, gridDim.x);
    for (int base = 0; base < a.n_items; base += gridDim.x) {
        const int it = base + local;
        if (it >= a.n_items) break;
        const int2 w = a.items[it];
        __syncthreads();  // the previous item's LDS reads are done
        spectrum_body<LOGM, LOGP, COUNTS, MONO, 1>(a, batch, w.y, w.x);
    }
}

template <int LOGM, int LOGP, bool COUNTS, bool MONO, int Q>
static void launch_spec_k(const SpecArgs& a, int blocks, int batch, hipStream_t st) {
    using C = SpecCfg<LOGM, Q>;
    const int groups = (batch + Q - 1) / Q;
    hipLaunchKernelGGL((k_spectrum<LOGM, LOGP, COUNTS, MONO, Q>), dim3(blocks, groups), dim3(C::WG), 0, st, a,
                       batch);
}

template <int LOGM, int LOGP, int Q>
static hipError_t launch_spec_t(const SpecArgs& a, int batch, hipStream_t st) {
    using C = SpecCfg<LOGM, Q>;
    const bool counts = a.flat != nullptr, mono = a.mono_part != nullptr;
    const int pairs = (a.V + 1) / 2;
    auto blocks = [&](int per) { return (pairs + C::FP * per - 1) / (C::FP * per); };
    if (counts && mono)
        launch_spec_k<LOGM, LOGP, true, true, Q>(a, blocks(spec_pairs<LOGP, true, true>()), batch, st);
    else if (counts)
        launch_spec_k<LOGM, LOGP, true, false, Q>(a, blocks(spec_pairs<LOGP, true, false>()), batch, st);
    else if (mono)
        launch_spec_k<LOGM, LOGP, false, true, Q>(a, blocks(spec_pairs<LOGP, false, true>()), batch, st);
    else
        launch_spec_k<LOGM, LOGP, false, false, Q>(a, blocks(spec_pairs<LOGP, false, false>()), batch, st);
    return hipGetLastError();
}

template <int LOGM, int Q>
static hipError_t launch_spec_q(const SpecArgs& a, int pr, int batch, hipStream_t st) {
    if constexpr (LOGM >= 4) {
        if (pr == 1) return launch_spec_t<LOGM, 0, Q>(a, batch, st);
    }
    if constexpr (LOGM >= 5) {
        if (pr == 2) return launch_spec_t<LOGM, 1, Q>(a, batch, st);
    }
    if constexpr (LOGM >= 6) {
        if (pr == 4) return launch_spec_t<LOGM, 2, Q>(a, batch, st);
    }
    return hipErrorInvalidValue;
}

template <int LOGM>
static hipError_t launch_spec_p(const SpecArgs& a, int pr, int q, int batch, hipStream_t st) {
    return q == 1 ? launch_spec_q<LOGM, 1>(a, pr, batch, st) : launch_spec_q<LOGM, kPolarSlices>(a, pr, batch, st);
}

// out[s][j][m] = polar sample m of projection j of slice s (diagnostics copy)
__global__ void __launch_bounds__(256) k_polar_extract(const float2* polar, float2* out, int V, int S, int lead,
                                                       int half_m, int q) {
    const int m = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y, s = blockIdx.z;
    if (m >= half_m) return;
    const int g = s / q, k = s % q;
    const PolarTiles lay{q, V, S};
    out[((size_t)s * V + j) * half_m + m] = polar[g * lay.group_elems() + lay.sample(j, lead + m) * q + k];
}

hipError_t launch_polar_extract(const bst_plan_s& p, const float2* polar, float2* out, int batch, hipStream_t st) {
    const int half_m = p.M / 2;
    hipLaunchKernelGGL(k_polar_extract, dim3((half_m + 255) / 256, p.V, batch), dim3(256), 0, st, polar, out, p.V,
                       p.S, p.lead, half_m, polar_group(p.taps));
    return hipGetLastError();
}

hipError_t launch_mass(const bst_plan_s& p, const MassArgs& a, int batch, hipStream_t st) {
    (void)p;
    const dim3 grid(kMassChunks, batch);
    if (a.flat != nullptr) hipLaunchKernelGGL(k_mass<true>, grid, dim3(kMassThreads), 0, st, a);
    else hipLaunchKernelGGL(k_mass<false>, grid, dim3(kMassThreads), 0, st, a);
    return hipGetLastError();
}

// ---- persistent launches (uneven batches: one slice per group) ----------------

template <int LOGM, int LOGP>
static hipError_t launch_spec_items_t(const SpecArgs& a, int batch, int blocks, hipStream_t st) {
    using C = SpecCfg<LOGM, 1>;
    if (a.mono_part)
        hipLaunchKernelGGL((k_spectrum_items<LOGM, LOGP, false, true>), dim3(blocks), dim3(C::WG), 0, st, a, batch);
    else
        hipLaunchKernelGGL((k_spectrum_items<LOGM, LOGP, false, false>), dim3(blocks), dim3(C::WG), 0, st, a, batch);
    return hipGetLastError();
}

template <int LOGM>
static hipError_t launch_spec_items_p(const SpecArgs& a, int pr, int batch, int blocks, hipStream_t st) {
    if constexpr (LOGM >= 4) {
        if (pr == 1) return launch_spec_items_t<LOGM, 0>(a, batch, blocks, st);
    }
    if constexpr (LOGM >= 5) {
        if (pr == 2) return launch_spec_items_t<LOGM, 1>(a, batch, blocks, st);
    }
    if constexpr (LOGM >= 6) {
        if (pr == 4) return launch_spec_items_t<LOGM, 2>(a, batch, blocks, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_spectrum_items(const bst_plan_s& p, const SpecArgs& a, int batch, int blocks, hipStream_t st) {
    if (a.flat) return hipErrorInvalidValue;  // raw counts are not batched
    const int pr = p.prm.pad_radial;
    switch (p.logM) {
        case 4: return launch_spec_items_p<4>(a, pr, batch, blocks, st);
        case 5: return launch_spec_items_p<5>(a, pr, batch, blocks, st);
        case 6: return launch_spec_items_p<6>(a, pr, batch, blocks, st);
        case 7: return launch_spec_items_p<7>(a, pr, batch, blocks, st);
        case 8: return launch_spec_items_p<8>(a, pr, batch, blocks, st);
        case 9: return launch_spec_items_p<9>(a, pr, batch, blocks, st);
        case 10: return launch_spec_items_p<10>(a, pr, batch, blocks, st);
        case 11: return launch_spec_items_p<11>(a, pr, batch, blocks, st);
        case 12: return launch_spec_items_p<12>(a, pr, batch, blocks, st);
        case 13: return launch_spec_items_p<13>(a, pr, batch, blocks, st);
        default: return hipErrorInvalidValue;
    }
}

template <int LOGM>
static int spec_blocks_t(int pr, bool mono, int V) {
    using C = SpecCfg<LOGM, 1>;
    const int per = (pr >= 2 && !mono) ? BST_SPEC_PAIRS : 1;  // as spec_pairs
    const int pairs = (V + 1) / 2;
    return (pairs + C::FP * per - 1) / (C::FP * per);
}

int spectrum_blocks_per_slice(const bst_plan_s& p, int V) {
    const int pr = p.prm.pad_radial;
    const bool mono = p.monopole;
    switch (p.logM) {
        case 4: return spec_blocks_t<4>(pr, mono, V);
        case 5: return spec_blocks_t<5>(pr, mono, V);
        case 6: return spec_blocks_t<6>(pr, mono, V);
        case 7: return spec_blocks_t<7>(pr, mono, V);
        case 8: return spec_blocks_t<8>(pr, mono, V);
        case 9: return spec_blocks_t<9>(pr, mono, V);
        case 10: return spec_blocks_t<10>(pr, mono, V);
        case 11: return spec_blocks_t<11>(pr, mono, V);
        case 12: return spec_blocks_t<12>(pr, mono, V);
        case 13: return spec_blocks_t<13>(pr, mono, V);
        default: return 0;
    }
}

hipError_t launch_spectrum(const bst_plan_s& p, const SpecArgs& a, int batch, hipStream_t st) {
    const int pr = p.prm.pad_radial;
    const int q = polar_group(p.taps);
    switch (p.logM) {
        case 4: return launch_spec_p<4>(a, pr, q, batch, st);
        case 5: return launch_spec_p<5>(a, pr, q, batch, st);
        case 6: return launch_spec_p<6>(a, pr, q, batch, st);
        case 7: return launch_spec_p<7>(a, pr, q, batch, st);
        case 8: return launch_spec_p<8>(a, pr, q, batch, st);
        case 9: return launch_spec_p<9>(a, pr, q, batch, st);
        case 10: return launch_spec_p<10>(a, pr, q, batch, st);
        case 11: return launch_spec_p<11>(a, pr, q, batch, st);
        case 12: return launch_spec_p<12>(a, pr, q, batch, st);
        case 13: return launch_spec_p<13>(a, pr, q, batch, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bst

BST_CHECK_MODULE(spectrum)
