// k_bruteforce.hip -- direct ("slant-stack") backprojection, Eq. 2 summed over
// the V angles, O(N^2 V) per slice (Section 2, last paragraph): the baseline
// the BST is measured against.
//
//   img[p][q] = sum_j w_j * sum_i y_j[i] Lambda(s - i),
//   s = n/2 + ((q - N/2) cos theta_j + (p - N/2) sin theta_j) * d/dt.
//
// A block owns a 32x32 pixel tile; each thread four consecutive pixels of one
// row. Angles are processed in chunks of 16: for each angle the block stages
// in LDS the 64 detector samples that the tile's footprint can touch (zero
// outside [0, n)), so the interpolation reads never leave LDS. The position
// s is formed in FP64 once per thread and angle (s reaches ~n, where FP32
// would leave ~1e-4 of error in the interpolation weight); the three
// neighbouring pixels step from it in FP32 within a few units, where FP32
// resolves the fraction to ~1e-7.
#include "bst_internal.h"

namespace bst {

constexpr int kTile = 32;
constexpr int kChunk = 16;
constexpr int kSeg = 64;

__global__ void __launch_bounds__(256) k_bruteforce(BfArgs a) {
    __shared__ float seg[kChunk][kSeg];
    __shared__ int seg_start[kChunk];
    const int tid = threadIdx.x;
    const int tx = tid & 7, ty = tid >> 3;
    const int q0 = blockIdx.x * kTile, p0 = blockIdx.y * kTile;
    const int s = blockIdx.z;
    const float* Y = a.sino + (size_t)s * a.V * a.n;
    const int half_n = a.N >> 1;
    const double X0 = (double)(q0 + 4 * tx - half_n);
    const double Yp = (double)(p0 + ty - half_n);
    const double cx0 = (double)(q0 - half_n), cx1 = (double)(q0 + kTile - 1 - half_n);
    const double cy0 = (double)(p0 - half_n), cy1 = (double)(p0 + kTile - 1 - half_n);
    const double sc = 0.5 * (double)a.n;
    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;

    for (int jc = 0; jc < a.V; jc += kChunk) {
        __syncthreads();
        if (tid < kChunk) {
            const int j = jc + tid;
            int st = 0;
            if (j < a.V) {
                const double c = a.c[j], sn = a.s[j];
                const double smin = sc + fmin(cx0 * c, cx1 * c) + fmin(cy0 * sn, cy1 * sn);
                st = (int)floor(smin) - 2;
            }
            seg_start[tid] = st;
        }
        __syncthreads();
        for (int l = tid; l < kChunk * kSeg; l += 256) {
            const int c = l / kSeg, o = l - c * kSeg;
            const int j = jc + c;
            const int i = seg_start[c] + o;
            seg[c][o] = (j < a.V && i >= 0 && i < a.n) ? Y[(size_t)j * a.n + i] : 0.f;
        }
        __syncthreads();
        const int cmax = min(kChunk, a.V - jc);
        for (int c = 0; c < cmax; ++c) {
            const int j = jc + c;
            const double cs = a.c[j], sn = a.s[j];
            const float w = a.w[j];
            const double sb = fma(X0, cs, fma(Yp, sn, sc));
            const double fl = floor(sb);
            const int ib = (int)fl - seg_start[c];
            const float fb = (float)(sb - fl);
            const float cf = (float)cs;
            const float* row = seg[c];
#define BST_BF_PIX(K, ACC)                                              \
            {                                                           \
                const float t = fmaf((float)(K), cf, fb);               \
                const float ft = floorf(t);                             \
                const int idx = ib + (int)ft;                           \
                const float fr = t - ft;                                \
                const float v0 = row[idx], v1 = row[idx + 1];           \
                ACC = fmaf(w, fmaf(fr, v1 - v0, v0), ACC);              \
            }
            BST_BF_PIX(0, acc0)
            BST_BF_PIX(1, acc1)
            BST_BF_PIX(2, acc2)
            BST_BF_PIX(3, acc3)
#undef BST_BF_PIX
        }
    }
    const int p = p0 + ty;
    const int q = q0 + 4 * tx;
    if (p < a.N) {
        float* o = a.img + ((size_t)s * a.N + p) * a.N;
        if (q + 0 < a.N) o[q + 0] = acc0;
        if (q + 1 < a.N) o[q + 1] = acc1;
        if (q + 2 < a.N) o[q + 2] = acc2;
        if (q + 3 < a.N) o[q + 3] = acc3;
    }
}

hipError_t launch_bruteforce(const bst_plan_s& p, const BfArgs& a, int batch, hipStream_t st) {
    (void)p;
    dim3 grid((a.N + kTile - 1) / kTile, (a.N + kTile - 1) / kTile, batch);
    hipLaunchKernelGGL(k_bruteforce, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace bst
