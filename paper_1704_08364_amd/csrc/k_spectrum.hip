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
// projection-pair groups per block: the next group's detector data is read
// while the current group is transformed
#ifndef BST_SPEC_PAIRS
#define BST_SPEC_PAIRS 2
#endif

namespace bst {

// Groups per block: the prefetch needs registers for one more group's data
// slots, which only the P_r >= 2 plain-input variants have to spare.
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
    const int lines = c < a.V ? (a.V - 1 - c) / kMassChunks + 1 : 0;
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
            float v = base[BST_IDX((size_t)(c + l * kMassChunks) * a.n + i, (size_t)a.V * a.n, 0)];
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

template <int LOGM>
struct SpecCfg {
    static constexpr int M = 1 << LOGM;
    static constexpr int T = M / 16;
    static constexpr int F = T >= 256 ? 1 : 256 / T;   // transforms (projection pairs) per block
    static constexpr int WG = F * T;
};

// LOGP = log2(P_r). Thread j's padded positions k = j + e*T hold data only for
// e < E0 or e >= 16 - E0 (E0 = 8 / P_r): the middle of every line is padding,
// known at compile time, so it is never loaded. COUNTS: the input is raw
// counts with per-slice flat and dark fields.
// Unpadded raw counts with the monopole hold the most per-thread state (16
// data slots and their flat and dark values): they get room for 3 waves per
// SIMD instead of spilling.
template <int LOGP, bool COUNTS, bool MONO>
constexpr int spec_waves() { return (MONO && COUNTS && LOGP == 0) ? 3 : BST_SPEC_WAVES; }

// MONO: monopole subtraction, y[i] - m phi[i] (m from the partial sums).
template <int LOGM, int LOGP, bool COUNTS, bool MONO>
__global__ void __launch_bounds__(SpecCfg<LOGM>::WG)
__attribute__((amdgpu_waves_per_eu(spec_waves<LOGP, COUNTS, MONO>(), 8))) k_spectrum(SpecArgs a) {
    using C = SpecCfg<LOGM>;
    constexpr int M = C::M, T = C::T;
    constexpr int E0 = 8 >> LOGP;
    constexpr int NQ = 2 * E0;  // data slots per thread
    __shared__ float2 lds[C::F * FftShape<LOGM>::LDS];
    const int fid = threadIdx.x / T;
    const int j = threadIdx.x - fid * T;
    float2* my = lds + fid * FftShape<LOGM>::LDS;
    const int s = blockIdx.y;
    const int h = a.n >> 1;
    constexpr int PAIRS = spec_pairs<LOGP, COUNTS, MONO>();
    const int npairs = (a.V + 1) >> 1;

    // detector bin of data slot q: positions e = q (q < E0) and e = 16 - 2*E0 + q (q >= E0)
    auto bin_of = [&](int q) {
        const int e = q < E0 ? q : 16 - 2 * E0 + q;
        const int k = j + e * T;
        return k < h ? k + h : k - M + h;
    };

    // Every global read of the thread is issued up front with no branch in
    // between: the data slots of both lines of the first group (a missing
    // line -- an odd V, or a group past the end -- reads line 0 and is
    // dropped by a select), the taper, flat and dark, the epilogue weights and
    // the twiddle anchors; these last are the same for every group.
    const float* base = a.sino_list ? a.sino_list[s] : a.sino + (size_t)s * a.V * a.n;
    auto load_lines = [&](int pair, float (&ra)[NQ], float (&rb)[NQ]) {
        const int ja = 2 * pair, jb = 2 * pair + 1;
        const float* ya = base + (size_t)(ja < a.V ? ja : 0) * a.n;
        const float* yb = base + (size_t)(jb < a.V ? jb : 0) * a.n;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int i = BST_IDX(bin_of(q), a.n, 1);
            ra[q] = ya[i];
            rb[q] = yb[i];
        }
    };
    float ra[NQ], rb[NQ], w[NQ];
    const int pair0 = blockIdx.x * PAIRS * C::F + fid;
    load_lines(pair0 < npairs ? pair0 : 0, ra, rb);
#pragma unroll
    for (int q = 0; q < NQ; ++q) w[q] = a.taper[bin_of(q)];
    float dk[COUNTS ? NQ : 1], fl[COUNTS ? NQ : 1];
    if constexpr (COUNTS) {
        const float* fs = a.flat + (size_t)s * a.n;
        const float* ds = a.dark + (size_t)s * a.n;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int i = bin_of(q);
            fl[q] = fs[i];
            dk[q] = ds[i];
        }
    }
    float mph[MONO ? NQ : 1];  // m phi at the thread's bins
    if constexpr (MONO) {
        const float m = monopole_mass(a.mono_part, s, a.mono_inv);
#pragma unroll
        for (int q = 0; q < NQ; ++q) mph[q] = m * a.mono_phi[bin_of(q)];
    }
    float2 kc[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) kc[e] = a.kc[j + e * T];
    const FftTwiddles<LOGM, -1, 16> tw(j, a.tw);

#pragma unroll
    for (int it = 0; it < PAIRS; ++it) {
        const int pair = pair0 + it * C::F;
        const int ja = 2 * pair, jb = 2 * pair + 1;
        const bool va = ja < a.V, vb = jb < a.V;
        float na[NQ], nb[NQ];
        if (it + 1 < PAIRS) {
            const int nx = pair + C::F;
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

        // fresh copies per group, so that nothing derived from them is
        // computed once and held across both transforms (that spills)
        FftTwiddles<LOGM, -1, 16> twl = tw;
        twl.pin();
        int jv = j;
        asm volatile("" : "+v"(jv));
        fft<LOGM, -1>(v, my, jv, twl);

#pragma unroll
        for (int e = 0; e < 16; ++e) my[lds_pad(jv + e * T)] = v[e];
        __syncthreads();

        float2* pa = a.polar + ((size_t)s * a.V + ja) * a.S;
        float2* pb = pa + a.S;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int m = jv + e * T;  // 0 .. M/2-1
            const float2 z = my[lds_pad(m)];
            const float2 zc = my[lds_pad((M - m) & (M - 1))];
            const float2 ya2 = cmul(make_float2(0.5f * (z.x + zc.x), 0.5f * (z.y - zc.y)), kc[e]);
            const float2 yb2 = cmul(make_float2(0.5f * (z.y + zc.y), -0.5f * (z.x - zc.x)), kc[e]);
            const int slot = BST_IDX(a.lead + m, a.S, 2);
            if (va) pa[slot] = ya2;
            if (vb) pb[slot] = yb2;
            // the sample before 0 (cubic radial taps): Yh(-sigma) = conj Yh(sigma)
            if (a.lead && m == 1) {
                if (va) pa[0] = make_float2(ya2.x, -ya2.y);
                if (vb) pb[0] = make_float2(yb2.x, -yb2.y);
            }
        }
        for (int z = jv; z < a.tail; z += T) {
            const int slot = BST_IDX(a.lead + M / 2 + z, a.S, 2);
            if (va) pa[slot] = make_float2(0.f, 0.f);
            if (vb) pb[slot] = make_float2(0.f, 0.f);
        }
        if (jv == 0) {
            const float2 z0 = my[0];
            if (va) a.dc[(size_t)s * a.V + BST_IDX(ja, a.V, 3)] = a.dt * z0.x;
            if (vb) a.dc[(size_t)s * a.V + BST_IDX(jb, a.V, 3)] = a.dt * z0.y;
        }
        if (it + 1 < PAIRS) {
            __syncthreads();  // the next transform overwrites this LDS
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                ra[q] = na[q];
                rb[q] = nb[q];
            }
        }
    }
}

template <int LOGM, int LOGP, bool COUNTS, bool MONO>
static void launch_spec_k(const SpecArgs& a, int groups, int batch, hipStream_t st) {
    using C = SpecCfg<LOGM>;
    constexpr int P = spec_pairs<LOGP, COUNTS, MONO>();
    hipLaunchKernelGGL((k_spectrum<LOGM, LOGP, COUNTS, MONO>), dim3((groups + P - 1) / P, batch), dim3(C::WG), 0,
                       st, a);
}

template <int LOGM, int LOGP>
static hipError_t launch_spec_t(const SpecArgs& a, int batch, hipStream_t st) {
    using C = SpecCfg<LOGM>;
    const int pairs = (a.V + 1) / 2;
    const int groups = (pairs + C::F - 1) / C::F;
    const bool counts = a.flat != nullptr, mono = a.mono_part != nullptr;
    if (counts && mono) launch_spec_k<LOGM, LOGP, true, true>(a, groups, batch, st);
    else if (counts) launch_spec_k<LOGM, LOGP, true, false>(a, groups, batch, st);
    else if (mono) launch_spec_k<LOGM, LOGP, false, true>(a, groups, batch, st);
    else launch_spec_k<LOGM, LOGP, false, false>(a, groups, batch, st);
    return hipGetLastError();
}

template <int LOGM>
static hipError_t launch_spec_p(const SpecArgs& a, int pr, int batch, hipStream_t st) {
    if constexpr (LOGM >= 4) {
        if (pr == 1) return launch_spec_t<LOGM, 0>(a, batch, st);
    }
    if constexpr (LOGM >= 5) {
        if (pr == 2) return launch_spec_t<LOGM, 1>(a, batch, st);
    }
    if constexpr (LOGM >= 6) {
        if (pr == 4) return launch_spec_t<LOGM, 2>(a, batch, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_mass(const bst_plan_s& p, const MassArgs& a, int batch, hipStream_t st) {
    (void)p;
    const dim3 grid(kMassChunks, batch);
    if (a.flat != nullptr) hipLaunchKernelGGL(k_mass<true>, grid, dim3(kMassThreads), 0, st, a);
    else hipLaunchKernelGGL(k_mass<false>, grid, dim3(kMassThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_spectrum(const bst_plan_s& p, const SpecArgs& a, int batch, hipStream_t st) {
    const int pr = p.prm.pad_radial;
    switch (p.logM) {
        case 4: return launch_spec_p<4>(a, pr, batch, st);
        case 5: return launch_spec_p<5>(a, pr, batch, st);
        case 6: return launch_spec_p<6>(a, pr, batch, st);
        case 7: return launch_spec_p<7>(a, pr, batch, st);
        case 8: return launch_spec_p<8>(a, pr, batch, st);
        case 9: return launch_spec_p<9>(a, pr, batch, st);
        case 10: return launch_spec_p<10>(a, pr, batch, st);
        case 11: return launch_spec_p<11>(a, pr, batch, st);
        case 12: return launch_spec_p<12>(a, pr, batch, st);
        case 13: return launch_spec_p<13>(a, pr, batch, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bst

BST_CHECK_MODULE(spectrum)
