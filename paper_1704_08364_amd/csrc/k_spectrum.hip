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
// load forms y = -log((I - D)/(I0 - D)) first (flat/dark normalisation). Output rows hold m = 0..M/2-1 plus two zero slots (row stride
// S = M/2 + 2) so the gather may read samples m0 and m0+1 without a bound test.
// The unweighted DC values dt*Y_j[0] go to a separate array for the origin rule.
#include "bst_internal.h"
#include "fft_lds.h"

namespace bst {

template <int LOGM>
struct SpecCfg {
    static constexpr int M = 1 << LOGM;
    static constexpr int T = M / 16;
    static constexpr int F = T >= 256 ? 1 : 256 / T;   // transforms (projection pairs) per block
    static constexpr int WG = F * T;
};

template <int LOGM>
__global__ void __launch_bounds__(SpecCfg<LOGM>::WG) k_spectrum(SpecArgs a) {
    using C = SpecCfg<LOGM>;
    constexpr int M = C::M, T = C::T;
    __shared__ float2 lds[C::F * FftShape<LOGM>::LDS];
    const int fid = threadIdx.x / T;
    const int j = threadIdx.x - fid * T;
    float2* my = lds + fid * FftShape<LOGM>::LDS;
    const int pair = blockIdx.x * C::F + fid;
    const int s = blockIdx.y;
    const int ja = 2 * pair, jb = 2 * pair + 1;
    const bool va = ja < a.V, vb = jb < a.V;
    const int h = a.n >> 1;
    const float* ya = a.sino + ((size_t)s * a.V + (va ? ja : 0)) * a.n;
    const float* yb = a.sino + ((size_t)s * a.V + (vb ? jb : 0)) * a.n;

    // raw counts: y = -log((I - D) / (I0 - D)) with the slice's flat/dark rows
    const float* fl = a.flat ? a.flat + (size_t)s * a.n : nullptr;
    const float* dk = a.flat ? a.dark + (size_t)s * a.n : nullptr;
    float2 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int k = j + e * T;
        const int i = (k < h) ? k + h : ((k >= M - h) ? k - M + h : -1);
        float x = 0.f, y = 0.f;
        if (i >= 0) {
            const float w = a.taper[i];
            float ra = va ? ya[i] : 0.f, rb = vb ? yb[i] : 0.f;
            if (fl) {
                const float d = dk[i], inv = 1.0f / (fl[i] - d);
                ra = va ? -logf((ra - d) * inv) : 0.f;
                rb = vb ? -logf((rb - d) * inv) : 0.f;
            }
            x = w * ra;
            y = w * rb;
        }
        v[e] = make_float2(x, y);
    }

    fft<LOGM, -1>(v, my, j, a.tw);

#pragma unroll
    for (int e = 0; e < 16; ++e) my[lds_pad(j + e * T)] = v[e];
    __syncthreads();

    float2* pa = a.polar + ((size_t)s * a.V + ja) * a.S;
    float2* pb = pa + a.S;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int m = j + e * T;  // 0 .. M/2-1
        const float2 z = my[lds_pad(m)];
        const float2 zc = my[lds_pad((M - m) & (M - 1))];
        const float2 kc = a.kc[m];
        const float2 ra = cmul(make_float2(0.5f * (z.x + zc.x), 0.5f * (z.y - zc.y)), kc);
        const float2 rb = cmul(make_float2(0.5f * (z.y + zc.y), -0.5f * (z.x - zc.x)), kc);
        if (va) pa[m] = ra;
        if (vb) pb[m] = rb;
    }
    if (j < 2) {
        if (va) pa[M / 2 + j] = make_float2(0.f, 0.f);
        if (vb) pb[M / 2 + j] = make_float2(0.f, 0.f);
    }
    if (j == 0) {
        const float2 z0 = my[0];
        if (va) a.dc[(size_t)s * a.V + ja] = a.dt * z0.x;
        if (vb) a.dc[(size_t)s * a.V + jb] = a.dt * z0.y;
    }
}

template <int LOGM>
static hipError_t launch_spec_t(const SpecArgs& a, int batch, hipStream_t st) {
    using C = SpecCfg<LOGM>;
    const int pairs = (a.V + 1) / 2;
    dim3 grid((pairs + C::F - 1) / C::F, batch);
    hipLaunchKernelGGL(k_spectrum<LOGM>, grid, dim3(C::WG), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_spectrum(const bst_plan_s& p, const SpecArgs& a, int batch, hipStream_t st) {
    switch (p.logM) {
        case 4: return launch_spec_t<4>(a, batch, st);
        case 5: return launch_spec_t<5>(a, batch, st);
        case 6: return launch_spec_t<6>(a, batch, st);
        case 7: return launch_spec_t<7>(a, batch, st);
        case 8: return launch_spec_t<8>(a, batch, st);
        case 9: return launch_spec_t<9>(a, batch, st);
        case 10: return launch_spec_t<10>(a, batch, st);
        case 11: return launch_spec_t<11>(a, batch, st);
        case 12: return launch_spec_t<12>(a, batch, st);
        case 13: return launch_spec_t<13>(a, batch, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bst
