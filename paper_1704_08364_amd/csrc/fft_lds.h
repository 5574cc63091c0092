// fft_lds.h -- in-register / LDS Stockham FFT used by every BST kernel.
//
// A transform of length L = 2^l is held by T = L/E threads (E = 8, 16 or 32);
// thread j keeps the E values x[j + e*T], e = 0..E-1, in registers on entry and
// X[j + e*T] on exit (natural order). With B = 3 for E = 8 and B = 4
// otherwise, passes are radix 2^(l mod B) first (if l is not a multiple of B)
// and then radix 2^B. Each pass computes its butterflies in registers;
// between passes the values go through LDS once (write, barrier, read, barrier).
// The Stockham auto-sort indexing (Govindaraju et al., SC'08) keeps every pass
// in natural order, so no bit reversal is needed.
//
// LDS layout: element i of a transform sits at position lds_swz<E>(i), an XOR
// swizzle (bits [0, B) of i XOR bits [B, 2B), bits [B, 2B) XOR bits [2B, 3B),
// B = log2 of the main radix). It is a permutation of [0, L) that is linear
// over the bits, so pos(a + b) = pos(a) ^ pos(b) when a and b share no set
// bit: a butterfly's R outputs and a thread's E inputs are one per-thread
// position XOR a compile-time constant. 8-byte LDS accesses on gfx950 are
// served 32 lanes at a time over 32 eight-byte banks for reads and 16 lanes
// at a time over 16 banks for writes (measured with SQ_LDS_BANK_CONFLICT);
// under that model every read and every write of the passes below touches
// distinct banks at the lengths of 2048-bin slices (L = 2048 and 4096; a few
// write conflicts remain at some shorter lengths), where a plain i + i/16
// padding costs two extra cycles on each contiguous read.
//
// A transform's region starts at a byte offset `off` of the block's LDS array
// that is a multiple of 8 L, so the region and the position OR together and
// the thread's byte offset of an element is one XOR with a constant (the
// instruction's offset field takes the array's address): one VALU operation
// per LDS access. The positions of a region are XOR-ed with a mask xm below L
// that puts transforms sharing a wave on different banks: region_xor for
// transforms interleaved lane by lane (thread t serves transform t mod F),
// contiguous_xor for transforms on contiguous ranges of threads.
//
// Inter-pass twiddles: one value w = tw[(jj mod NS) * L/(NS R)] per butterfly
// from a table tw[k] = exp(-2 pi i k / L) computed in FP64 on the host and
// rounded to FP32; the other powers w^r are products of its squarings (at most
// six roundings deep), which replaces R-1 scattered table reads by one
// coalesced read. The inverse direction conjugates them. The anchors of all
// passes are read together before the first pass (FftTwiddles), so no pass
// waits on a table read, and a thread that runs many transforms of one length
// can read them once and keep them in registers.
#pragma once

#include <hip/hip_runtime.h>

namespace bst {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// multiply by exp(DIR * i * pi / 2): -i for the forward (DIR = -1), +i for the inverse
template <int DIR>
__device__ __forceinline__ float2 rot90(float2 a) {
    return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}
// multiply by c + DIR * i * s
template <int DIR>
__device__ __forceinline__ float2 cmulc(float2 a, float c, float s) {
    const float sd = DIR < 0 ? -s : s;
    return make_float2(fmaf(a.x, c, -a.y * sd), fmaf(a.x, sd, a.y * c));
}

template <int E>
__host__ __device__ constexpr int lds_swz(int i) {
    constexpr int B = E >= 16 ? 4 : 3;
    constexpr int M = (1 << B) - 1;
    return i ^ ((i >> B) & M) ^ (((i >> (2 * B)) & M) << B);
}

// Byte offset of position p of the region at byte `off` with mask xm.
__device__ __forceinline__ unsigned lds_byte(unsigned off, int p, int xm) {
    return off | ((unsigned)(p ^ xm) << 3);
}
// The byte XOR of element offset c (no bit in common with the thread's part).
template <int E>
__host__ __device__ constexpr unsigned swz_bytes(int c) {
    return (unsigned)lds_swz<E>(c) << 3;
}
// The float2 at byte offset b of the block's LDS array.
__device__ __forceinline__ float2& lds_at(float2* lds, unsigned b) {
    return *reinterpret_cast<float2*>(reinterpret_cast<char*>(lds) + b);
}

// Mask of transform f of F interleaved lane by lane, linear in the bits of f
// (per-bit masks from the bank model; bits of f past the fourth reuse none).
template <int LOGL, int F>
__device__ __forceinline__ int region_xor(int f) {
    int m = 0;
    if constexpr (F == 2) {
        m = f ? 24 : 0;
    } else if constexpr (F == 4) {
        m = ((f & 1) ? 8 : 0) ^ ((f & 2) ? 20 : 0);
    } else if constexpr (F == 8) {
        m = ((f & 1) ? 4 : 0) ^ ((f & 2) ? 8 : 0) ^ ((f & 4) ? 18 : 0);
    } else if constexpr (F >= 16) {
        m = ((f & 1) ? 16 : 0) ^ ((f & 2) ? 4 : 0) ^ ((f & 4) ? 6 : 0) ^ ((f & 8) ? 8 : 0);
    }
    return m & ((1 << LOGL) - 1);  // any mask below L keeps the region
}
// Mask of transform u of transforms on contiguous ranges of T threads: those
// sharing a 32-lane half then sit on disjoint banks.
template <int LOGL, int T>
__device__ __forceinline__ int contiguous_xor(int u) {
    return T >= 32 ? 0 : ((u * T) & 31 & ((1 << LOGL) - 1));
}

constexpr float kC1 = 0.92387953251128675613f;  // cos(pi/8)
constexpr float kS1 = 0.38268343236508977173f;  // sin(pi/8)
constexpr float kH = 0.70710678118654752440f;   // cos(pi/4)

template <int DIR>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
    const float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
    const float2 t0 = cadd(x0, x2), t1 = csub(x0, x2);
    const float2 t2 = cadd(x1, x3), t3 = rot90<DIR>(csub(x1, x3));
    x0 = cadd(t0, t2);
    x2 = csub(t0, t2);
    x1 = cadd(t1, t3);
    x3 = csub(t1, t3);
}

// natural order in, natural order out
template <int DIR>
__device__ __forceinline__ void dft8(float2* v) {
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<DIR>(e0, e1, e2, e3);
    dft4<DIR>(o0, o1, o2, o3);
    o1 = cmulc<DIR>(o1, kH, kH);
    o2 = rot90<DIR>(o2);
    o3 = cmulc<DIR>(o3, -kH, kH);
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

template <int DIR>
__device__ __forceinline__ void dft16(float2* v) {
    float2 e[8], o[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) { e[i] = v[2 * i]; o[i] = v[2 * i + 1]; }
    dft8<DIR>(e);
    dft8<DIR>(o);
    o[1] = cmulc<DIR>(o[1], kC1, kS1);
    o[2] = cmulc<DIR>(o[2], kH, kH);
    o[3] = cmulc<DIR>(o[3], kS1, kC1);
    o[4] = rot90<DIR>(o[4]);
    o[5] = cmulc<DIR>(o[5], -kS1, kC1);
    o[6] = cmulc<DIR>(o[6], -kH, kH);
    o[7] = cmulc<DIR>(o[7], -kC1, kS1);
#pragma unroll
    for (int k = 0; k < 8; ++k) { v[k] = cadd(e[k], o[k]); v[k + 8] = csub(e[k], o[k]); }
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v) {
    if constexpr (R == 2) dft2<DIR>(v[0], v[1]);
    else if constexpr (R == 4) dft4<DIR>(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8<DIR>(v);
    else dft16<DIR>(v);
}

// One Stockham pass of radix R over sub-transforms of size NS (product of the
// earlier radices). Butterfly jj (= j + k*T) reads x[jj + r*L/R] -- which is
// v[k + r*(16/R)] in this thread's registers -- twiddles it by
// w^((jj mod NS) * r) with w = exp(DIR 2 pi i / (NS R)), transforms, and
// writes output r to position (jj / NS) * NS * R + (jj mod NS) + r * NS.
// anc[k]: the twiddle anchor of butterfly k, already conjugated for DIR > 0
template <int L, int DIR, int R, int NS, int E>
__device__ __forceinline__ void stockham_pass(float2 (&v)[E], float2* lds, unsigned off, int j, const float2* anc,
                                              int xm) {
    constexpr int T = L / E;
    constexpr int BPT = E / R;
    constexpr bool LAST = (NS * R == L);
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int jj = j + k * T;
        float2 x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = v[k + r * BPT];
        if constexpr (NS > 1) {
            // one table anchor w per butterfly; w^r is the product of the
            // anchor's binary powers w, w^2, w^4, w^8 picked by the bits of r
            // (at most three products after at most three squarings), formed
            // just before use so that few twiddles are live at once
            const float2 w1 = anc[k];
            float2 w2 = w1, w4 = w1, w8 = w1;
            if constexpr (R >= 4) w2 = cmul(w1, w1);
            if constexpr (R >= 8) w4 = cmul(w2, w2);
            if constexpr (R >= 16) w8 = cmul(w4, w4);
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w;
                bool first = true;
                if (r & 1) { w = w1; first = false; }
                if (r & 2) { w = first ? w2 : cmul(w, w2); first = false; }
                if (r & 4) { w = first ? w4 : cmul(w, w4); first = false; }
                if (r & 8) { w = first ? w8 : cmul(w, w8); }
                x[r] = cmul(x[r], w);
            }
        }
        dft<R, DIR>(x);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[k + r * BPT] = x[r];
        } else {
            const unsigned pb = lds_byte(off, lds_swz<E>((jj / NS) * NS * R + (jj & (NS - 1))), xm);
#pragma unroll
            for (int r = 0; r < R; ++r) lds_at(lds, pb ^ swz_bytes<E>(r * NS)) = x[r];
        }
    }
    if constexpr (!LAST) {
        __syncthreads();
        const unsigned pj = lds_byte(off, lds_swz<E>(j), xm);
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = lds_at(lds, pj ^ swz_bytes<E>(e * T));
        __syncthreads();
    }
}

// Twiddle anchors of every pass of one transform of length 2^LOGL held by
// threads with E values each (the pass plan of fft below): w[p][k] belongs to
// butterfly k of the p-th pass that has twiddles (the first pass has none).
template <int LOGL, int DIR, int E>
struct FftTwiddles {
    static constexpr int L = 1 << LOGL;
    static constexpr int T = L / E;
    static constexpr int LR = E >= 16 ? 4 : 3;           // log2 of the main radix
    static constexpr int R = 1 << LR;
    static constexpr int REM = LOGL % LR;
    static constexpr int NS0 = REM != 0 ? (1 << REM) : R;  // NS of the first twiddled pass
    static constexpr int BPT = E / R;
    static constexpr int count() {
        int c = 0;
        for (int ns = NS0; ns < L; ns *= R) ++c;
        return c;
    }
    static constexpr int NT = count();
    float2 w[NT > 0 ? NT : 1][BPT];

    __device__ __forceinline__ FftTwiddles(int j, const float2* __restrict__ tw) {
#pragma unroll
        for (int p = 0; p < NT; ++p) {
            const int ns = NS0 << (LR * p);
#pragma unroll
            for (int k = 0; k < BPT; ++k) {
                const int m = (j + k * T) & (ns - 1);
                float2 x = tw[m * (L / (ns * R))];
                if constexpr (DIR > 0) x.y = -x.y;
                w[p][k] = x;
            }
        }
    }

    // Make the anchors opaque to the optimiser at this point. A caller that
    // runs one transform per loop iteration with loop-invariant anchors calls
    // this on a copy inside the loop; otherwise every derived power w^r is
    // hoisted out of the loop and held in registers for its whole length.
    __device__ __forceinline__ void pin() {
#pragma unroll
        for (int p = 0; p < NT; ++p) {
#pragma unroll
            for (int k = 0; k < BPT; ++k) asm volatile("" : "+v"(w[p][k].x), "+v"(w[p][k].y));
        }
    }
};

template <int LOGL, int DIR, int R, int NS, int E, int P>
__device__ __forceinline__ void radix_passes(float2 (&v)[E], float2* lds, unsigned off, int j,
                                             const FftTwiddles<LOGL, DIR, E>& tw, int xm) {
    constexpr int L = 1 << LOGL;
    if constexpr (NS < L) {
        stockham_pass<L, DIR, R, NS, E>(v, lds, off, j, tw.w[P], xm);
        radix_passes<LOGL, DIR, R, NS * R, E, (NS > 1 ? P + 1 : P)>(v, lds, off, j, tw, xm);
    }
}

// Full transform of length 2^LOGL by L/E threads holding E (8, 16 or 32)
// values each; passes are radix min(E, 16) after one smaller first pass when
// needed. Requires every thread of the block to call it (barriers); `lds` is
// the block's LDS array, and the transform's region of L float2 at byte `off`
// (a multiple of 8 L; positions lds_swz<E>(i) ^ xm) must not be read by
// anyone else meanwhile. Ends with a barrier if any LDS exchange happened.
template <int LOGL, int DIR, int E = 16>
__device__ __forceinline__ void fft(float2 (&v)[E], float2* lds, unsigned off, int j,
                                    const FftTwiddles<LOGL, DIR, E>& tw, int xm) {
    static_assert(E == 8 || E == 16 || E == 32, "8, 16 or 32 values per thread");
    using TW = FftTwiddles<LOGL, DIR, E>;
    constexpr int L = 1 << LOGL;
    if constexpr (TW::REM != 0) {
        stockham_pass<L, DIR, (1 << TW::REM), 1, E>(v, lds, off, j, tw.w[0], xm);
        radix_passes<LOGL, DIR, TW::R, (1 << TW::REM), E, 0>(v, lds, off, j, tw, xm);
    } else {
        radix_passes<LOGL, DIR, TW::R, 1, E, 0>(v, lds, off, j, tw, xm);
    }
}

// The same, reading the twiddle anchors from the table first.
template <int LOGL, int DIR, int E = 16>
__device__ __forceinline__ void fft(float2 (&v)[E], float2* lds, unsigned off, int j, const float2* __restrict__ tw,
                                    int xm) {
    const FftTwiddles<LOGL, DIR, E> t(j, tw);
    fft<LOGL, DIR, E>(v, lds, off, j, t, xm);
}

// Blocks of a 1D grid are dispatched round-robin over the 8 XCDs of an
// MI355X (block b runs on XCD b mod 8), each with its own L2. This maps the
// hardware block index to a logical one so that every XCD receives one
// contiguous range of logical blocks, and neighbouring logical blocks -- which
// read neighbouring data -- share an L2.
__device__ __forceinline__ int xcd_contiguous(int bid, int nblocks) {
    constexpr int kXcd = 8;
    const int per = nblocks / kXcd, rem = nblocks % kXcd;
    const int x = bid % kXcd, k = bid / kXcd;
    return x * per + (x < rem ? x : rem) + k;
}

}  // namespace bst
