// Host check of the hand-written reverse derivatives (mhd_adjoint.hpp)
// against forward-mode dual numbers through the same physics header
// (mhd_physics.hpp instantiated on an 8-direction dual type): for random
// states covering the HLLD fan regions, B_n = 0, identical states, B_perp = 0
// and the limiter cases, J^T a from the reverse code must equal the
// contraction of the dual-number Jacobian with a.  Test infrastructure only.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <algorithm>
#include <cstdlib>
#define __host__
#define __device__
#define __forceinline__ inline
#define VLCT_HOST_COUNT
#include "mhd_adjoint.hpp"

namespace vlct_ad {
constexpr int kDir = 8;
struct D8 {
    double v;
    double d[kDir];
    constexpr D8(double x = 0.0) : v(x), d{} {}
};
inline D8 operator+(const D8 &a, const D8 &b) { D8 r(a.v + b.v); for (int k = 0; k < kDir; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
inline D8 operator-(const D8 &a, const D8 &b) { D8 r(a.v - b.v); for (int k = 0; k < kDir; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
inline D8 operator-(const D8 &a) { D8 r(-a.v); for (int k = 0; k < kDir; ++k) r.d[k] = -a.d[k]; return r; }
inline D8 operator*(const D8 &a, const D8 &b) { D8 r(a.v * b.v); for (int k = 0; k < kDir; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
inline D8 operator/(const D8 &a, const D8 &b) { const double q = a.v / b.v; D8 r(q); for (int k = 0; k < kDir; ++k) r.d[k] = (a.d[k] - q * b.d[k]) / b.v; return r; }
inline bool operator<(const D8 &a, const D8 &b) { return a.v < b.v; }
inline bool operator>(const D8 &a, const D8 &b) { return a.v > b.v; }
inline bool operator<=(const D8 &a, const D8 &b) { return a.v <= b.v; }
inline bool operator>=(const D8 &a, const D8 &b) { return a.v >= b.v; }
inline bool operator==(const D8 &a, const D8 &b) { return a.v == b.v; }
inline bool operator!=(const D8 &a, const D8 &b) { return a.v != b.v; }
inline D8 sqrt(const D8 &a) { const double s = std::sqrt(a.v); D8 r(s); const double h = s > 0.0 ? 0.5 / s : 0.0; for (int k = 0; k < kDir; ++k) r.d[k] = a.d[k] * h; return r; }
inline D8 fabs(const D8 &a) { D8 r = a.v < 0.0 ? -a : a; r.v = std::fabs(a.v); return r; }
inline D8 fmin(const D8 &a, const D8 &b) { return b.v < a.v ? b : a; }
inline D8 fmax(const D8 &a, const D8 &b) { return b.v > a.v ? b : a; }
inline D8 copysign(const D8 &a, const D8 &b) { const bool flip = std::signbit(a.v) != std::signbit(b.v); return flip ? -a : a; }
#define double D8
#include "phys_copy.hpp"
#undef double
}  // namespace vlct_ad

using vlct::W7;
namespace P = vlct_ad::vlct;
using vlct_ad::D8;

static std::mt19937_64 rng(12345);
static double U(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

static W7 rand_w(double vs) {
    return W7{U(0.2, 3.0), U(-vs, vs), U(-2, 2), U(-2, 2), U(0.05, 3.0), U(-2, 2), U(-2, 2)};
}
static void w_arr(const W7 &w, double x[7]) { x[0]=w.d; x[1]=w.u; x[2]=w.v; x[3]=w.w; x[4]=w.p; x[5]=w.by; x[6]=w.bz; }

int main(int argc, char **argv) {
    const int trials = argc > 1 ? atoi(argv[1]) : 20000;
    const double gam = 5.0 / 3.0, gm1i = 1.0 / (gam - 1.0);
    double worst = 0; int nbad = 0;
    for (int trial = 0; trial < trials; ++trial) {
        const double vs = trial % 4 == 0 ? 8.0 : 2.0;
        W7 L = rand_w(vs), R = rand_w(vs);
        double bn = trial % 7 == 0 ? 0.0 : U(-2, 2);
        if (trial % 11 == 0) R = L;  // identical states
        double lf[7]; for (auto &x : lf) x = U(-1, 1);
        W7 aL{0,0,0,0,0,0,0}, aR{0,0,0,0,0,0,0}; double abn = 0;
        vlct::hlld_rev(L, R, bn, gam, gm1i, lf, aL, aR, abn);
        double x[15]; w_arr(L, x); w_arr(R, x + 7); x[14] = bn;
        double g[16];
        for (int pass = 0; pass < 2; ++pass) {
            D8 in[15];
            for (int q = 0; q < 15; ++q) { in[q] = D8(x[q]); int kk = q - pass * 8; if (kk >= 0 && kk < 8) in[q].d[kk] = 1.0; }
            P::W7 wl{in[0],in[1],in[2],in[3],in[4],in[5],in[6]}, wr{in[7],in[8],in[9],in[10],in[11],in[12],in[13]};
            D8 f[7], upw;
            P::hlld(wl, wr, in[14], D8(gam), D8(gm1i), f, upw);
            for (int kk = 0; kk < 8; ++kk) { double s = 0; for (int c = 0; c < 7; ++c) s += lf[c] * f[c].d[kk]; if (pass*8+kk < 16) g[pass*8+kk] = s; }
        }
        double got[15]; w_arr(aL, got); w_arr(aR, got + 7); got[14] = abn;
        double sc = 0; for (int q = 0; q < 15; ++q) sc = std::max(sc, std::fabs(g[q]));
        for (int q = 0; q < 15; ++q) {
            double e = std::fabs(got[q] - g[q]) / (sc + 1e-300);
            if (e > worst) worst = e;
            if (e > 1e-10) { if (nbad < 10) printf("hlld trial %d input %d: rev %.15g dual %.15g\n", trial, q, got[q], g[q]); nbad++; }
        }
    }
    printf("HLLD: worst rel err %.3e, bad %d\n", worst, nbad);

    for (int chr = 0; chr < 2; ++chr) {
        worst = 0; nbad = 0;
        for (int trial = 0; trial < trials; ++trial) {
            W7 w0 = rand_w(2.0);
            auto pert = [&](double s) { W7 w = w0; w.d *= 1 + U(-s, s); w.u += U(-s, s); w.v += U(-s, s); w.w += U(-s, s); w.p *= 1 + U(-s, s); w.by += U(-s, s); w.bz += U(-s, s); return w; };
            double s = trial % 3 == 0 ? 0.02 : 0.3;
            W7 wm = pert(s), wp = pert(s);
            double bn = trial % 9 == 0 ? 0.0 : U(-2, 2);
            if (trial % 13 == 0) { w0.by = 0; w0.bz = 0; }
            double afm[7], afp[7]; for (auto &v : afm) v = U(-1, 1); for (auto &v : afp) v = U(-1, 1);
            W7 am{0,0,0,0,0,0,0}, a0{0,0,0,0,0,0,0}, ap{0,0,0,0,0,0,0}; double abn = 0;
            if (chr) vlct::plmc_rev<true>(wm, w0, wp, bn, gam, afm, afp, am, a0, ap, abn);
            else vlct::plmc_rev<false>(wm, w0, wp, bn, gam, afm, afp, am, a0, ap, abn);
            double x[22]; w_arr(wm, x); w_arr(w0, x + 7); w_arr(wp, x + 14); x[21] = bn;
            double g[24];
            for (int pass = 0; pass < 3; ++pass) {
                D8 in[22];
                for (int q = 0; q < 22; ++q) { in[q] = D8(x[q]); int kk = q - pass * 8; if (kk >= 0 && kk < 8) in[q].d[kk] = 1.0; }
                P::W7 a{in[0],in[1],in[2],in[3],in[4],in[5],in[6]}, b{in[7],in[8],in[9],in[10],in[11],in[12],in[13]}, c{in[14],in[15],in[16],in[17],in[18],in[19],in[20]};
                P::W7 fm, fp;
                if (chr) P::plmc<true>(a, b, c, in[21], D8(gam), fm, fp); else P::plmc<false>(a, b, c, in[21], D8(gam), fm, fp);
                const D8 *o[14] = {&fm.d,&fm.u,&fm.v,&fm.w,&fm.p,&fm.by,&fm.bz,&fp.d,&fp.u,&fp.v,&fp.w,&fp.p,&fp.by,&fp.bz};
                for (int kk = 0; kk < 8; ++kk) { double s2 = 0; for (int c2 = 0; c2 < 7; ++c2) s2 += afm[c2] * o[c2]->d[kk] + afp[c2] * o[7+c2]->d[kk]; if (pass*8+kk < 24) g[pass*8+kk] = s2; }
            }
            double got[22]; w_arr(am, got); w_arr(a0, got + 7); w_arr(ap, got + 14); got[21] = abn;
            double sc = 0; for (int q = 0; q < 22; ++q) sc = std::max(sc, std::fabs(g[q]));
            for (int q = 0; q < 22; ++q) {
                double e = std::fabs(got[q] - g[q]) / (sc + 1e-300);
                if (e > worst) worst = e;
                if (e > 1e-10) { if (nbad < 10) printf("plmc%d trial %d input %d: rev %.15g dual %.15g\n", chr, trial, q, got[q], g[q]); nbad++; }
            }
        }
        printf("PLM%s: worst rel err %.3e, bad %d\n", chr ? "C" : "P", worst, nbad);
    }

    // PPMC / PPMP over five-cell stencils: random ones (extremum and
    // overshoot branches, the bounds), smooth ones (the unlimited parabola),
    // stencils with repeated cells (the tie snapping) and B_n = 0
    for (int chr = 0; chr < 2; ++chr) {
        worst = 0; nbad = 0;
        for (int trial = 0; trial < trials; ++trial) {
            W7 w0 = rand_w(2.0);
            W7 st[5];
            const int kind = trial % 4;
            if (kind == 1) {
                // smooth profile: w0 + k g + k^2 h with small g, h
                double gx[7], hx[7];
                for (int c = 0; c < 7; ++c) { gx[c] = U(-0.05, 0.05); hx[c] = U(-0.01, 0.01); }
                for (int k = -2; k <= 2; ++k) {
                    double x[7]; w_arr(w0, x);
                    for (int c = 0; c < 7; ++c) x[c] += k * gx[c] + k * k * hx[c];
                    st[k + 2] = W7{x[0], x[1], x[2], x[3], x[4], x[5], x[6]};
                }
            } else {
                const double s = kind == 2 ? 0.02 : 0.3;
                for (int k = 0; k < 5; ++k) {
                    W7 w = w0;
                    w.d *= 1 + U(-s, s); w.u += U(-s, s); w.v += U(-s, s); w.w += U(-s, s);
                    w.p *= 1 + U(-s, s); w.by += U(-s, s); w.bz += U(-s, s);
                    st[k] = w;
                }
                st[2] = w0;
                if (kind == 3) { st[0] = st[1]; st[4] = w0; }  // repeated cells
            }
            double bn = trial % 9 == 0 ? 0.0 : U(-2, 2);
            if (trial % 13 == 0) { for (auto &w : st) { w.by = 0; w.bz = 0; } }
            double afm[7], afp[7]; for (auto &v : afm) v = U(-1, 1); for (auto &v : afp) v = U(-1, 1);
            W7 a[5]; for (auto &w : a) w = W7{0,0,0,0,0,0,0}; double abn = 0;
            if (chr) vlct::ppmc_rev<true>(st[0], st[1], st[2], st[3], st[4], bn, gam, afm, afp, a[0], a[1], a[2], a[3], a[4], abn);
            else vlct::ppmc_rev<false>(st[0], st[1], st[2], st[3], st[4], bn, gam, afm, afp, a[0], a[1], a[2], a[3], a[4], abn);
            double x[36]; for (int k = 0; k < 5; ++k) w_arr(st[k], x + 7 * k); x[35] = bn;
            double g[40];
            for (int pass = 0; pass < 5; ++pass) {
                D8 in[36];
                for (int q = 0; q < 36; ++q) { in[q] = D8(x[q]); int kk = q - pass * 8; if (kk >= 0 && kk < 8) in[q].d[kk] = 1.0; }
                P::W7 w[5];
                for (int k = 0; k < 5; ++k) w[k] = P::W7{in[7*k],in[7*k+1],in[7*k+2],in[7*k+3],in[7*k+4],in[7*k+5],in[7*k+6]};
                P::W7 fm, fp;
                if (chr) P::ppmc<true>(w[0], w[1], w[2], w[3], w[4], in[35], D8(gam), fm, fp);
                else P::ppmc<false>(w[0], w[1], w[2], w[3], w[4], in[35], D8(gam), fm, fp);
                const D8 *o[14] = {&fm.d,&fm.u,&fm.v,&fm.w,&fm.p,&fm.by,&fm.bz,&fp.d,&fp.u,&fp.v,&fp.w,&fp.p,&fp.by,&fp.bz};
                for (int kk = 0; kk < 8; ++kk) { double s2 = 0; for (int c2 = 0; c2 < 7; ++c2) s2 += afm[c2] * o[c2]->d[kk] + afp[c2] * o[7+c2]->d[kk]; if (pass*8+kk < 40) g[pass*8+kk] = s2; }
            }
            double got[36]; for (int k = 0; k < 5; ++k) w_arr(a[k], got + 7 * k); got[35] = abn;
            double sc = 0; for (int q = 0; q < 36; ++q) sc = std::max(sc, std::fabs(g[q]));
            for (int q = 0; q < 36; ++q) {
                double e = std::fabs(got[q] - g[q]) / (sc + 1e-300);
                if (e > worst) worst = e;
                if (e > 1e-10) { if (nbad < 10) printf("ppmc%d trial %d input %d: rev %.15g dual %.15g\n", chr, trial, q, got[q], g[q]); nbad++; }
            }
        }
        printf("PPM%s: worst rel err %.3e, bad %d\n", chr ? "C" : "P", worst, nbad);
    }
    return 0;
}
