// k_bruteforce.hip -- direct ("slant-stack") backprojection, Eq. 2 summed over
// the V angles, O(N^2 V) per slice (Section 2, last paragraph): the baseline
// the BST is measured against.
//
//   img[p][q] = sum_j w_j * sum_i y_j[i] Lambda(s - i),
//   s = n/2 + ((q - N/2) cos theta_j + (p - N/2) sin theta_j) * d/dt.
//
// The kernel is bound by vector ALU issue (one interpolate-accumulate per
// pixel and angle), so it is written to spend few instructions per pair:
//   - a block owns a 64 x 32 pixel tile, each thread eight consecutive
//     pixels of one row, so the per-angle position set-up (FP64) is shared by
//     eight interpolations;
//   - angles go in chunks of 16; for each angle the block stages in LDS the
//     detector samples the tile's footprint can touch as pairs
//     (w_j y[i], w_j (y[i+1] - y[i])) (zero outside [0, n)), so one 8-byte
//     LDS read gives both the value and the slope, already weighted;
//   - per pixel: position u = f + k cos (FP32, u > 0 by an offset of 8, so
//     truncation is the floor), index and fraction, one LDS read, and
//     acc += A + fract(u) D.
// The position of the thread's first pixel is formed in FP64 (s reaches ~n,
// where FP32 would leave ~1e-4 of error in the weight); the other seven step
// from its fraction in FP32 within 16 units, where FP32 resolves the fraction
// to ~1e-6.
#include "bst_internal.h"

namespace bst {

constexpr int kTileX = 64;   // pixels per tile row (8 threads x 8 pixels)
constexpr int kTileY = 32;   // tile rows
constexpr int kPix = 8;      // consecutive pixels per thread
constexpr int kChunk = 16;   // angles staged together
// Detector samples staged per angle. The tile's positions s span at most
// sqrt(63^2 + 31^2) < 70.3 bins (d/dt = 1: n_out == n_det), so floor(s) of
// any pixel is at most 71 above floor(s_min); the segment starts kPix + 1
// below floor(s_min) (the positions' offset, and FP32 rounding of the
// first pixel's fraction to 1), so the entries read lie in [1, 81].
constexpr int kSeg = 88;

__global__ void __launch_bounds__(256) k_bruteforce(BfArgs a) {
    __shared__ float2 seg[kChunk * kSeg];
    __shared__ int seg_start[kChunk];
    __shared__ double2 dir[kChunk];  // (cos, sin) * d/dt of the chunk's angles
    const int tid = threadIdx.x;
    const int tx = tid & 7, ty = tid >> 3;
    const int q0 = blockIdx.x * kTileX, p0 = blockIdx.y * kTileY;
    const int s = blockIdx.z;
    const float* Y = a.sino + (size_t)s * a.V * a.n;
    const int half_n = a.N >> 1;
    const double X0 = (double)(q0 + kPix * tx - half_n);
    const double Yp = (double)(p0 + ty - half_n);
    const double cx0 = (double)(q0 - half_n), cx1 = (double)(q0 + kTileX - 1 - half_n);
    const double cy0 = (double)(p0 - half_n), cy1 = (double)(p0 + kTileY - 1 - half_n);
    const double sc = 0.5 * (double)a.n;
    float acc[kPix];
#pragma unroll
    for (int k = 0; k < kPix; ++k) acc[k] = 0.f;

    for (int jc = 0; jc < a.V; jc += kChunk) {
        __syncthreads();
        if (tid < kChunk) {
            const int j = jc + tid;
            int st = 0;
            double c = 0.0, sn = 0.0;
            if (j < a.V) {
                c = a.c[j];
                sn = a.s[j];
                const double smin = sc + fmin(cx0 * c, cx1 * c) + fmin(cy0 * sn, cy1 * sn);
                // kPix + 1 below the footprint: the positions carry an offset of kPix
                st = (int)floor(smin) - 1 - kPix;
            }
            seg_start[tid] = st;
            dir[tid] = make_double2(c, sn);
        }
        __syncthreads();
        for (int l = tid; l < kChunk * kSeg; l += 256) {
            const int c = l / kSeg, o = l - c * kSeg;
            const int j = jc + c;
            const int i = seg_start[c] + o;
            float y0 = 0.f, y1 = 0.f, w = 0.f;
            if (j < a.V) {
                w = a.w[j];
                if (i >= 0 && i < a.n) y0 = Y[(size_t)j * a.n + i];
                if (i + 1 >= 0 && i + 1 < a.n) y1 = Y[(size_t)j * a.n + i + 1];
            }
            seg[l] = make_float2(w * y0, w * (y1 - y0));
        }
        __syncthreads();
        const int cmax = min(kChunk, a.V - jc);
        for (int c = 0; c < cmax; ++c) {
            const double2 cs = dir[c];
            const double sb = fma(X0, cs.x, fma(Yp, cs.y, sc));
            const double fl = floor(sb);
            // this thread's entries: sample floor(s) of its first pixel sits at
            // index base + kPix, pixel k's sample at base + (int)u
            int base = c * kSeg + (int)fl - kPix - seg_start[c];
            // formed once per angle (otherwise its terms are re-added per pixel)
            asm volatile("" : "+v"(base));
            const float fb = (float)(sb - fl) + (float)kPix;
            const float cf = (float)cs.x;
#pragma unroll
            for (int k = 0; k < kPix; ++k) {
                const float u = fmaf((float)k, cf, fb);  // in [1, 17)
                const float2 e = seg[base + (int)u];
                acc[k] += fmaf(__builtin_amdgcn_fractf(u), e.y, e.x);
            }
        }
    }
    const int p = p0 + ty;
    if (p < a.N) {
        float* o = a.img + ((size_t)s * a.N + p) * a.N;
#pragma unroll
        for (int k = 0; k < kPix; ++k) {
            const int q = q0 + kPix * tx + k;
            if (q < a.N) o[q] = acc[k];
        }
    }
}

// Ramp filter of the brute-force FBP: the band-limited spatial kernel of Kak
// and Slaney sampled at the detector pitch, applied as a linear (not circular)
// convolution, q[i] = dt sum_k h[i - k] y[k] over the n bins. Only d = 0 and
// odd distances d carry weight. One block per projection; the row is staged
// in LDS in FP64 and every output sums its terms in FP64 in a fixed order.
constexpr int kRampThreads = 256;

__global__ void __launch_bounds__(kRampThreads) k_ramp_filter(RampArgs a) {
    extern __shared__ double row[];
    const int j = blockIdx.x, s = blockIdx.y;
    const float* y = a.sino + ((size_t)s * a.V + j) * a.n;
    for (int i = threadIdx.x; i < a.n; i += kRampThreads) row[i] = (double)y[i];
    __syncthreads();
    float* q = a.out + ((size_t)s * a.V + j) * a.n;
    for (int i = threadIdx.x; i < a.n; i += kRampThreads) {
        double acc = a.h[0] * row[i];
        // odd distances d: the samples i - d and i + d that exist
        for (int d = 1; d < a.n; d += 2) {
            const double l = i - d >= 0 ? row[i - d] : 0.0;
            const double r = i + d < a.n ? row[i + d] : 0.0;
            acc = fma(a.h[d], l + r, acc);
        }
        q[i] = (float)acc;
    }
}

hipError_t launch_ramp_filter(const bst_plan_s& p, const RampArgs& a, int batch, hipStream_t st) {
    (void)p;
    hipLaunchKernelGGL(k_ramp_filter, dim3(a.V, batch), dim3(kRampThreads), a.n * sizeof(double), st, a);
    return hipGetLastError();
}

hipError_t launch_bruteforce(const bst_plan_s& p, const BfArgs& a, int batch, hipStream_t st) {
    // the LDS segment length assumes one detector bin per pixel (d == dt)
    if (p.n != p.N) return hipErrorInvalidValue;
    dim3 grid((a.N + kTileX - 1) / kTileX, (a.N + kTileY - 1) / kTileY, batch);
    hipLaunchKernelGGL(k_bruteforce, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace bst
