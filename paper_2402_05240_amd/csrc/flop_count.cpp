// flop_count.cpp -- counts the FP64 arithmetic of the device physics per call
// (PLMC reconstruction, PPMC reconstruction, HLLD solve, and their reverse
// derivatives used by the adjoint) by compiling the same source on the host
// with a counting scalar.  Convention: one FLOP per add,
// subtract, multiply, divide or square root; comparisons, min, max, abs and
// copysign count zero.  Branch-dependent paths are averaged over random
// turbulence-like states (rho ~ 1, |v| ~ 1, P ~ 0.6, B ~ (1.1, 0, 0) + 0.2 noise).
//
// Build and run:  g++ -O1 -std=c++17 -o /tmp/flop_count flop_count.cpp && /tmp/flop_count
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>

static long long g_flops = 0;

struct Counted {
    double v;
    constexpr Counted(double x = 0.0) : v(x) {}
};
#define BIN(OP)                                                                              \
    inline Counted operator OP(Counted a, Counted b) { ++g_flops; return Counted(a.v OP b.v); } \
    inline Counted operator OP(double a, Counted b) { ++g_flops; return Counted(a OP b.v); }    \
    inline Counted operator OP(Counted a, double b) { ++g_flops; return Counted(a.v OP b); }
BIN(+) BIN(-) BIN(*) BIN(/)
#undef BIN
inline Counted operator-(Counted a) { return Counted(-a.v); }
#define CMP(OP)                                                                   \
    inline bool operator OP(Counted a, Counted b) { return a.v OP b.v; }          \
    inline bool operator OP(Counted a, double b) { return a.v OP b; }             \
    inline bool operator OP(double a, Counted b) { return a OP b.v; }
CMP(<) CMP(>) CMP(<=) CMP(>=) CMP(==) CMP(!=)
#undef CMP
inline Counted sqrt(Counted a) { ++g_flops; return Counted(std::sqrt(a.v)); }
inline Counted fabs(Counted a) { return Counted(std::fabs(a.v)); }
inline Counted fmin(Counted a, Counted b) { return Counted(std::fmin(a.v, b.v)); }
inline Counted fmax(Counted a, Counted b) { return Counted(std::fmax(a.v, b.v)); }
inline Counted fmin(Counted a, double b) { return Counted(std::fmin(a.v, b)); }
inline Counted fmax(Counted a, double b) { return Counted(std::fmax(a.v, b)); }
inline Counted copysign(Counted a, Counted b) { return Counted(std::copysign(a.v, b.v)); }
inline Counted copysign(double a, Counted b) { return Counted(std::copysign(a, b.v)); }

#define VLCT_HOST_COUNT
#define double Counted
#include "mhd_physics.hpp"
#include "mhd_adjoint.hpp"
#undef double

int main()
{
    std::mt19937_64 rng(2402), rng_cot(5240);
    std::normal_distribution<double> nrm(0.0, 1.0);
    std::uniform_real_distribution<double> uni(0.8, 1.2);
    const double gam = 5.0 / 3.0, gm1i = 1.0 / (gam - 1.0);
    auto state = [&]() {
        return vlct::W7{uni(rng), nrm(rng), nrm(rng), nrm(rng), 0.6 * uni(rng), 0.2 * nrm(rng),
                        0.2 * nrm(rng)};
    };
    const int N = 20000;
    long long plmc_f = 0, ppmc_f = 0, plmp_f = 0, ppmp_f = 0, hlld_f = 0;
    long long hlld_r = 0, plmc_r = 0, plmp_r = 0, ppmc_r = 0, ppmp_r = 0;
    for (int q = 0; q < N; ++q) {
        vlct::W7 a = state(), b = state(), c = state(), d = state(), e = state();
        // smooth-ish stencils: neighbours close to the centre
        auto mix = [&](const vlct::W7 &x, const vlct::W7 &y, double t) {
            return vlct::W7{x.d.v + t * (y.d.v - x.d.v), x.u.v + t * (y.u.v - x.u.v),
                            x.v.v + t * (y.v.v - x.v.v), x.w.v + t * (y.w.v - x.w.v),
                            x.p.v + t * (y.p.v - x.p.v), x.by.v + t * (y.by.v - x.by.v),
                            x.bz.v + t * (y.bz.v - x.bz.v)};
        };
        vlct::W7 m2 = mix(c, a, 0.2), m1 = mix(c, b, 0.1), p1 = mix(c, d, 0.1), p2 = mix(c, e, 0.2);
        const double bn = 1.1 + 0.2 * nrm(rng);
        vlct::W7 fm, fp;
        long long f0 = g_flops;
        vlct::plmc<true>(m1, c, p1, Counted(bn), Counted(gam), fm, fp);
        plmc_f += g_flops - f0;
        f0 = g_flops;
        vlct::ppmc<true>(m2, m1, c, p1, p2, Counted(bn), Counted(gam), fm, fp);
        ppmc_f += g_flops - f0;
        f0 = g_flops;
        vlct::plmc<false>(m1, c, p1, Counted(bn), Counted(gam), fm, fp);
        plmp_f += g_flops - f0;
        f0 = g_flops;
        vlct::ppmc<false>(m2, m1, c, p1, p2, Counted(bn), Counted(gam), fm, fp);
        ppmp_f += g_flops - f0;
        Counted f[7], upw;
        f0 = g_flops;
        vlct::hlld(m1, c, Counted(bn), Counted(gam), Counted(gm1i), f, upw);
        hlld_f += g_flops - f0;
        // reverse derivatives (the adjoint's per-face and per-cell maps)
        Counted af[7], afm[7], afp[7];
        for (int k = 0; k < 7; ++k) {
            af[k] = Counted(nrm(rng_cot));
            afm[k] = Counted(nrm(rng_cot));
            afp[k] = Counted(nrm(rng_cot));
        }
        vlct::W7 aL{0, 0, 0, 0, 0, 0, 0}, aR{0, 0, 0, 0, 0, 0, 0}, a3{0, 0, 0, 0, 0, 0, 0};
        Counted abn(0.0);
        f0 = g_flops;
        vlct::hlld_rev(m1, c, Counted(bn), Counted(gam), Counted(gm1i), af, aL, aR, abn);
        hlld_r += g_flops - f0;
        f0 = g_flops;
        vlct::plmc_rev<true>(m1, c, p1, Counted(bn), Counted(gam), afm, afp, aL, aR, a3, abn);
        plmc_r += g_flops - f0;
        f0 = g_flops;
        vlct::plmc_rev<false>(m1, c, p1, Counted(bn), Counted(gam), afm, afp, aL, aR, a3, abn);
        plmp_r += g_flops - f0;
        vlct::W7 a4{0, 0, 0, 0, 0, 0, 0}, a5{0, 0, 0, 0, 0, 0, 0};
        f0 = g_flops;
        vlct::ppmc_rev<true>(m2, m1, c, p1, p2, Counted(bn), Counted(gam), afm, afp, aL, aR, a3,
                             a4, a5, abn);
        ppmc_r += g_flops - f0;
        f0 = g_flops;
        vlct::ppmc_rev<false>(m2, m1, c, p1, p2, Counted(bn), Counted(gam), afm, afp, aL, aR, a3,
                              a4, a5, abn);
        ppmp_r += g_flops - f0;
    }
    std::printf("plmc_per_call %.1f\nppmc_per_call %.1f\nhlld_per_call %.1f\n",
                double(plmc_f) / N, double(ppmc_f) / N, double(hlld_f) / N);
    // a corrector face needs one reconstruction (each cell's reconstruction
    // serves its two faces) and one HLLD solve
    std::printf("plmp_per_call %.1f\nppmp_per_call %.1f\n", double(plmp_f) / N,
                double(ppmp_f) / N);
    std::printf("plmc_hlld_per_face %.1f\nppmc_hlld_per_face %.1f\n",
                double(plmc_f + hlld_f) / N, double(ppmc_f + hlld_f) / N);
    std::printf("plmp_hlld_per_face %.1f\nppmp_hlld_per_face %.1f\n",
                double(plmp_f + hlld_f) / N, double(ppmp_f + hlld_f) / N);
    // adjoint: a corrector face reverses HLLD at interface states recomputed
    // by one reconstruction per cell (row and march kernels; the first,
    // cell-parallel version recomputed two per face); every cell reverses its
    // reconstruction; a predictor face reverses HLLD on the cell states
    std::printf("hlld_rev_per_call %.1f\nplmc_rev_per_call %.1f\nplmp_rev_per_call %.1f\n",
                double(hlld_r) / N, double(plmc_r) / N, double(plmp_r) / N);
    std::printf("adj_faces_plmc_per_face %.1f (cell-parallel: %.1f)\nadj_faces_pcm_per_face %.1f\n",
                double(plmc_f + hlld_r) / N, double(2 * plmc_f + hlld_r) / N,
                double(hlld_r) / N);
    std::printf("adj_march_fused_plmc_per_cell %.1f\n",
                double(plmc_f + hlld_r + plmc_r) / N);
    // fused predictor, per cell: three PCM HLLD solves (its low x-, y- and
    // z-faces) and, counted by hand from the kernel's source, 195 more:
    // primitives 27 (B_cc 6, one division, v 3, kinetic 7, magnetic 6,
    // pressure 4), reference field 9, three edge fields 3 x 17 (mean 4, four
    // upwind terms 8, sum 5), cell update 5 x 9, face update 3 x 6, and the
    // half-step primitives 45 (three high faces 18, B_cc 6, the rest 21)
    std::printf("predictor_per_cell %.1f\n", 3.0 * double(hlld_f) / N + 195.0);
    std::printf("ppmc_rev_per_call %.1f\nppmp_rev_per_call %.1f\n", double(ppmc_r) / N,
                double(ppmp_r) / N);
    std::printf("adj_faces_ppmc_per_face %.1f (cell-parallel: %.1f)\n",
                double(ppmc_f + hlld_r) / N, double(2 * ppmc_f + hlld_r) / N);
    return 0;
}
