// plan_adjoint.cpp -- host construction of the transposed gather used by
// bst_project: for every polar sample (j, m), m < M/2, the list of Cartesian
// half-plane points (a, b) whose stencil (step P5 of Section 2) reads it,
// with the stencil weight and the conjugation flag. Coordinates are formed in
// FP64 with the same rules as the forward gather: radius index
// r = |(a,b)| P_r/P_c; direction theta = atan2(b, a) (plus pi and conjugation
// below the k_x axis), bracketed in the period-pi continuation of the angle
// sequence (uniform: q = theta V/pi; otherwise the last angle <= theta, the
// image theta_{V-1} - pi below theta_0, theta_0 + pi past theta_{V-1}, images
// conjugated); radial taps m0, m0+1 (linear) or m0-1 .. m0+2 with the Keys
// weights (a = -1/2), a tap at m < 0 read as the conjugate of -m; samples
// m >= M/2 zero; the origin and the Nyquist column k_x = G/2 excluded (they
// have their own rules). Lists are filled in increasing point order, so the
// device sum has a fixed order.
//
// The tent angular rule (an option of P5, uniform angles, linear radial taps)
// replaces the two bracketing angles of a point at Cartesian radius
// rho < V/pi by every angle index j of the period-pi continuation with
// |q - j| < h, h = V/(pi rho), weighted (1 - |q - j|/h) and normalised; index
// j + V is the conjugated image of angle j. These "wide" points are
// enumerated column by column (column a holds rows |b| <= B_a, the origin
// slot included but left empty); the forward gather evaluates their taps on
// the device, and the transposed lists of bst_project take the same taps.
#include <algorithm>
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

namespace {

// Keys cubic convolution weight (a = -1/2) at distance x
double keys_weight(double x) {
    x = std::fabs(x);
    if (x <= 1.0) return (1.5 * x - 2.5) * x * x + 1.0;
    if (x < 2.0) return ((-0.5 * x + 2.5) * x - 4.0) * x + 2.0;
    return 0.0;
}

struct Tap {
    int j;
    bool flip;
    double w;
};

// Tent taps of direction th in [0, pi) at Cartesian radius rho >= 1 (h > 1).
void tent_taps(double th, double rho, int V, std::vector<Tap>& out) {
    out.clear();
    const double q = th * ((double)V / M_PI);
    const double h = (double)V / (M_PI * rho);
    const long lo = (long)std::floor(q - h), hi = (long)std::ceil(q + h);
    double total = 0.0;
    for (long jc = lo; jc <= hi; ++jc) {
        const double w = 1.0 - std::fabs(q - (double)jc) / h;
        if (w <= 0.0) continue;
        long wraps = jc >= 0 ? jc / V : -((-jc + V - 1) / V);  // floor(jc / V)
        const int j = (int)(jc - wraps * (long)V);
        out.push_back({j, (wraps & 1) != 0, w});
        total += w;
    }
    for (auto& t : out) t.w /= total;
}

}  // namespace

size_t tent_columns(int G, int V, std::vector<int2>& cols) {
    // wide points: a^2 + b^2 < (V/pi)^2 (where the tent is wider than one step)
    const double R = (double)V / M_PI;
    cols.assign(G / 2, make_int2(0, -1));
    size_t total = 0;
    for (int a = 0; a < G / 2; ++a) {
        int B = -1;
        if ((double)a < R) {
            B = (int)std::floor(std::sqrt(std::max(0.0, R * R - (double)a * a)));
            while (B >= 0 && (double)a * a + (double)B * B >= R * R) --B;
            B = std::min(B, G / 2 - 1);
        }
        cols[a] = make_int2((int)total, B);
        if (B >= 0) total += (size_t)(2 * B + 1);
    }
    return total;
}

void tent_chunks(int V, const std::vector<int2>& cols, std::vector<int4>& chunks, std::vector<int>& coff) {
    chunks.clear();
    size_t W = 0;
    for (const auto& c : cols)
        if (c.y >= 0) W = (size_t)c.x + 2 * (size_t)c.y + 1;
    coff.assign(W + 1, 0);
    for (int a = 0; a < (int)cols.size(); ++a) {
        const int B = cols[a].y;
        for (int b = -B; b <= B; ++b) {
            const size_t idx = (size_t)cols[a].x + (size_t)(b + B);
            if (!(a == 0 && b == 0)) {
                // the tap range of the point, one index wider on each side than
                // |q - j| < h needs (taps outside it get weight 0 on the device)
                const double rho = std::sqrt((double)a * a + (double)b * b);
                const double phi = std::atan2((double)b, (double)a);
                const double q = (phi < 0.0 ? phi + M_PI : phi) * ((double)V / M_PI);
                const double h = (double)V / (M_PI * rho);
                const int lo = (int)std::floor(q - h) - 1, hi = (int)std::ceil(q + h) + 1;
                for (int j0 = lo; j0 <= hi; j0 += kTentChunk)
                    chunks.push_back(make_int4((int)idx, j0, std::min(hi, j0 + kTentChunk - 1), 0));
            }
            coff[idx + 1] = (int)chunks.size();
        }
    }
}

int tent_rows(int V, int M, double rscale) {
    // wide points have rho < V/pi, so radial taps m0 <= floor(rscale V/pi) and m0 + 1
    const int rows = (int)std::floor(rscale * (double)V / M_PI) + 2;
    return std::min(rows, M / 2);
}

bool build_adjoint_tables(int V, int M, int G, double rscale, const std::vector<double>& theta, bool uniform,
                          int taps, const std::vector<int2>* tent_cols, std::vector<int>& off,
                          std::vector<uint2>& ent) {
    const int Mh = M / 2;
    const size_t samples = (size_t)V * Mh;
    off.assign(samples + 1, 0);
    std::vector<StencilEntry> tmp;
    tmp.reserve((size_t)G * G * (taps / 2));  // ~ 2*taps entries x (G/2 x G) x pi/4
    for (int a = 0; a < G / 2; ++a) {
        for (int bi = 0; bi < G; ++bi) {
            const int b = bi < G / 2 ? bi : bi - G;
            if (a == 0 && b == 0) continue;
            const double r = std::sqrt((double)a * a + (double)b * b) * rscale;
            if (r >= (double)Mh + (taps == 4 ? 1.0 : 0.0)) continue;
            const double phi = std::atan2((double)b, (double)a);
            const bool lower = phi < 0.0;
            const double th = lower ? phi + M_PI : phi;
            const uint32_t pt = (uint32_t)a * (uint32_t)G + (uint32_t)bi;
            const double rho = std::sqrt((double)a * a + (double)b * b);
            if (tent_cols && std::abs(b) <= (*tent_cols)[a].y) {
                // wide point: the tent taps, linear radial taps
                std::vector<Tap> tt;
                tent_taps(th, rho, V, tt);
                const double mf = std::floor(r);
                const double g = r - mf;
                const int m0 = (int)mf;
                for (const auto& t : tt) {
                    const bool c = lower != t.flip;
                    for (int k = 0; k < 2; ++k) {
                        const int m = m0 + k;
                        const double w = t.w * (k ? g : 1.0 - g);
                        if (m >= Mh || w == 0.0) continue;
                        const int smp = t.j * Mh + m;
                        tmp.push_back({smp, pt | (c ? 0x80000000u : 0u), (float)w});
                        off[smp + 1]++;
                    }
                }
                continue;
            }
            int j0;
            double f;
            bool flip0 = false;
            if (uniform) {
                const double q = th * ((double)V / M_PI);
                const double qf = std::floor(q);
                f = q - qf;
                j0 = (int)qf;
                if (j0 >= V) { j0 = V - 1; f = 1.0; }
            } else {
                // last theta_j <= th; below theta_0 the image theta_{V-1} - pi
                const int k = (int)(std::upper_bound(theta.begin(), theta.end(), th) - theta.begin()) - 1;
                double lo, hi;
                if (k < 0) {
                    j0 = V - 1;
                    flip0 = true;
                    lo = theta[V - 1] - M_PI;
                    hi = theta[0];
                } else {
                    j0 = k;
                    lo = theta[k];
                    hi = (k + 1 < V) ? theta[k + 1] : theta[0] + M_PI;
                }
                f = (th - lo) / (hi - lo);
            }
            int j1 = j0 + 1;
            const bool wrap = (j1 == V);
            if (wrap) j1 = 0;
            const bool c0 = lower != flip0;
            const bool c1 = lower != (wrap && !flip0);
            const double mf = std::floor(r);
            const double g = r - mf;
            const int m0 = (int)mf;
            const int first = (taps == 4) ? -1 : 0;
            for (int side = 0; side < 2; ++side) {
                const int j = side ? j1 : j0;
                const double wa = side ? f : 1.0 - f;
                const bool c = side ? c1 : c0;
                for (int t = 0; t < taps; ++t) {
                    const int off_m = first + t;
                    const double wr = (taps == 4) ? keys_weight(g - off_m) : (off_m == 0 ? 1.0 - g : g);
                    int m = m0 + off_m;
                    bool cc = c;
                    if (m < 0) { m = -m; cc = !cc; }
                    const double w = wa * wr;
                    if (m >= Mh || w == 0.0) continue;
                    const int smp = j * Mh + m;
                    tmp.push_back({smp, pt | (cc ? 0x80000000u : 0u), (float)w});
                    off[smp + 1]++;
                }
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
