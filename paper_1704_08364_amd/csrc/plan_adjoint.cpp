// plan_adjoint.cpp -- host construction of the transposed gather used by
// bst_project: for every polar sample (j, m), m < M/2, the list of Cartesian
// half-plane points (a, b) whose bilinear stencil (step P5 of Section 2)
// reads it, with the stencil weight and the conjugation flag. Coordinates are
// formed in FP64 with the same rules as the forward gather: radius index
// r = |(a,b)| P_r/P_c, angle index q = theta V/pi with theta = atan2(b, a)
// (plus pi and conjugation below the k_x axis), neighbour past theta_{V-1} =
// theta_0 with the conjugation flipped, samples m >= M/2 zero, the origin
// excluded (it has its own rule). Lists are filled in increasing point order,
// so the device sum has a fixed order.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "bst_internal.h"

namespace bst {

struct StencilEntry {
    int sample;      // j * (M/2) + m
    uint32_t point;  // a * G + b | conj << 31
    float w;
};

bool build_adjoint_tables(int V, int M, int G, double rscale, std::vector<int>& off,
                          std::vector<uint2>& ent) {
    const int Mh = M / 2;
    const size_t samples = (size_t)V * Mh;
    off.assign(samples + 1, 0);
    std::vector<StencilEntry> tmp;
    tmp.reserve((size_t)G * G);  // ~ 4 entries x (G/2 x G) x pi/4
    for (int a = 0; a < G / 2; ++a) {
        for (int bi = 0; bi < G; ++bi) {
            const int b = bi < G / 2 ? bi : bi - G;
            if (a == 0 && b == 0) continue;
            const double r = std::sqrt((double)a * a + (double)b * b) * rscale;
            if (r >= (double)Mh) continue;
            const double phi = std::atan2((double)b, (double)a);
            const bool lower = phi < 0.0;
            const double th = lower ? phi + M_PI : phi;
            const double q = th * ((double)V / M_PI);
            double qf = std::floor(q);
            double f = q - qf;
            int j0 = (int)qf;
            if (j0 >= V) { j0 = V - 1; f = 1.0; }
            int j1 = j0 + 1;
            const bool wrap = (j1 == V);
            if (wrap) j1 = 0;
            const double mf = std::floor(r);
            const double g = r - mf;
            const int m0 = (int)mf;
            const uint32_t pt = (uint32_t)a * (uint32_t)G + (uint32_t)bi;
            const struct { int j, m; double w; bool c; } e4[4] = {
                {j0, m0, (1 - f) * (1 - g), lower},
                {j0, m0 + 1, (1 - f) * g, lower},
                {j1, m0, f * (1 - g), lower != wrap},
                {j1, m0 + 1, f * g, lower != wrap},
            };
            for (const auto& e : e4) {
                if (e.m >= Mh || e.w == 0.0) continue;
                const int smp = e.j * Mh + e.m;
                tmp.push_back({smp, pt | (e.c ? 0x80000000u : 0u), (float)e.w});
                off[smp + 1]++;
            }
        }
    }
    for (size_t i = 0; i < samples; ++i) off[i + 1] += off[i];
    ent.resize(tmp.size());
    std::vector<int> cursor(off.begin(), off.end() - 1);
    for (const auto& e : tmp) {
        uint32_t wbits;
        std::memcpy(&wbits, &e.w, 4);
        ent[cursor[e.sample]++] = make_uint2(e.point, wbits);
    }
    return true;
}

}  // namespace bst
