// mhd_physics.hpp -- per-state ideal-MHD physics on gfx950 for the VL+CT step
// (Caddy & Schneider, "Cholla-MHD", Sec. 2.1-2.2): wave speeds, the HLLD
// Riemann solver, the characteristic eigen-system and the PLMC / PPMC
// reconstructions.  Everything is FP64 and inlined into the kernels.
//
// Sweep frame: a 1D problem along axis d uses the state
//   W7 = (rho, v_n, v_t1, v_t2, P, B_t1, B_t2)
// with (n, t1, t2) the cyclic permutation (x,y,z), (y,z,x), (z,x,y) of the
// axes (Table emf and its note); the normal field B_n is a parameter.
#pragma once
#ifndef VLCT_HOST_COUNT
#include <hip/hip_runtime.h>
#define VLCT_DEV __device__ __forceinline__
#else
#define VLCT_DEV inline  // host build of the same code for operation counting
#endif

namespace vlct {

#ifndef VLCT_HOST_COUNT
// Square root of a finite argument >= 0 in the normal range (every use here:
// densities, pressures, squared speeds and field magnitudes, never subnormal
// or near overflow): the hardware reciprocal square root refined by one
// Goldschmidt step and two Newton corrections (Markstein's iteration), within
// an ulp of the correctly rounded root; zero maps to itself.  The library's
// sqrt differs only by the range scaling around the same iteration, which
// these arguments never need.
VLCT_DEV double msqrt(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    g = fma(d, h, g);
    return x == 0.0 ? x : g;  // rsq(0) is infinite
}
// Reciprocal square root of a finite argument > 0 in the normal range: the
// hardware estimate refined by two Newton steps y <- y + y (1 - x y^2) / 2
// (each doubles the correct bits of the estimate), within about an ulp.
// One of these replaces a square root and a division where both the root and
// its reciprocal are needed.
VLCT_DEV double mrsqrt(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double r = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, r, y);
    r = fma(-x * y, y, 1.0);
    return fma(0.5 * y, r, y);
}
#else
VLCT_DEV double msqrt(double x) { return sqrt(x); }
VLCT_DEV double mrsqrt(double x) { return 1.0 / sqrt(x); }
#endif

// Floors on derived and reconstructed rho, P (the conserved state is never changed).
constexpr double kFloorRho = 1.0e-20;
constexpr double kFloorP = 1.0e-20;
// HLLD: star states fall back to the outer states where
// |rho (S - u)(S - S_M) - B_n^2| < kHlldDegen * p_T*.
constexpr double kHlldDegen = 1.0e-8;
// Eigenvectors: B_n with |B_n| <= kBperpTiny sqrt(gP + B^2) is taken as zero and
// |B_perp| <= kBperpTiny sqrt(gP + B^2) uses beta_t1 = beta_t2 = 1/sqrt(2);
// rho (c_f^2 - c_s^2) <= kCfCsTiny rho c_f^2 uses alpha_f = 1, alpha_s = 0.
constexpr double kBperpTiny = 1.0e-12;
constexpr double kCfCsTiny = 1.0e-12;
// CT upwinding: |S_M| <= kUpwindTiny (c_max + |u_L| + |u_R|) counts as zero.
constexpr double kUpwindTiny = 1.0e-12;
// Colella-Sekora curvature ratio used by the PPMC limiters.
constexpr double kPpmC = 1.25;
// PPMC: a stencil difference below this fraction of the values' magnitudes (with
// c_f and sqrt(rho) c_f as floors for velocity and field components) is zero.
constexpr double kPpmTie = 1.0e-12;

constexpr uint32_t kStatusPressureFloor = 1u;
constexpr uint32_t kStatusDensityFloor = 2u;
constexpr uint32_t kStatusNonfinite = 4u;

struct W7 {
    double d, u, v, w, p, by, bz;
};

// Squared fast speed and the discriminant d = rho (c_f^2 - c_s^2) of the
// fast/slow speed formula (Sec. 2.2 Step 1), with the discriminant written as
// (gP - B^2)^2 + 4 gP B_perp^2 so it never cancels.
VLCT_DEV double fast_sq(double d, double p, double bn, double bt1, double bt2,
                                          double gam, double &disc)
{
    const double gp = gam * p;
    const double bp2 = bt1 * bt1 + bt2 * bt2;
    const double b2 = bn * bn + bp2;
    const double t = gp - b2;
    disc = msqrt(t * t + 4.0 * gp * bp2);
    return (gp + b2 + disc) / (2.0 * d);
}

VLCT_DEV double fast_speed(double d, double p, double bn, double bt1,
                                             double bt2, double gam)
{
    double disc;
    return msqrt(fast_sq(d, p, bn, bt1, bt2, gam, disc));
}

// ---------------------------------------------------------------------------
// HLLD (Sec. 2.2 Step 3, Miyoshi & Kusano 2005): 7 flux components in the
// sweep frame plus the CT upwind indicator (+1, -1, 0) taken from the sign of
// the interface (contact) velocity S_M, the sign of the mass flux.
// ---------------------------------------------------------------------------
VLCT_DEV void hlld(const W7 &L, const W7 &R, double bn, double gam, double gm1i,
                                     double f[7], double &upw)
{
    const double bn2 = bn * bn;
    const double pbL = 0.5 * (bn2 + L.by * L.by + L.bz * L.bz);
    const double pbR = 0.5 * (bn2 + R.by * R.by + R.bz * R.bz);
    const double ptL = L.p + pbL;
    const double ptR = R.p + pbR;
    const double eL = L.p * gm1i + 0.5 * L.d * (L.u * L.u + L.v * L.v + L.w * L.w) + pbL;
    const double eR = R.p * gm1i + 0.5 * R.d * (R.u * R.u + R.v * R.v + R.w * R.w) + pbR;
    // c_f = sqrt(num / (2 rho)) = num / sqrt(2 rho num), num = gP + B^2 + disc
    // (the fast-speed formula of fast_sq with one reciprocal root per side)
    auto fast = [&](const W7 &X) {
        const double gp = gam * X.p;
        const double bp2 = X.by * X.by + X.bz * X.bz;
        const double b2 = bn2 + bp2;
        const double t = gp - b2;
        const double num = gp + b2 + msqrt(t * t + 4.0 * gp * bp2);
        return num * mrsqrt(2.0 * X.d * num);
    };
    const double cfL = fast(L);
    const double cfR = fast(R);
    const double cmax = fmax(cfL, cfR);
    const double sL = fmin(L.u, R.u) - cmax;
    const double sR = fmax(L.u, R.u) + cmax;

    const double qL = (sL - L.u) * L.d;
    const double qR = (sR - R.u) * R.d;
    const double iq = 1.0 / (qR - qL);
    const double sM = (qR * R.u - qL * L.u - ptR + ptL) * iq;
    const double pts = (qR * ptL - qL * ptR + qL * qR * (R.u - L.u)) * iq;

    // single-star states of both sides (the energy only where it is used,
    // on the side whose fan contains x/t = 0)
    double ds[2], vs[2], ws[2], bys[2], bzs[2], issm[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const W7 &X = a == 0 ? L : R;
        const double S = a == 0 ? sL : sR;
        const double su = S - X.u;
        const double ssm = S - sM;
        issm[a] = 1.0 / ssm;
        ds[a] = X.d * su * issm[a];
        const double den = X.d * su * ssm - bn2;
        const bool degen = fabs(den) < kHlldDegen * pts;
        const double iden = 1.0 / den;
        const double t1 = degen ? 0.0 : bn * (sM - X.u) * iden;
        const double t2 = degen ? 1.0 : (X.d * su * su - bn2) * iden;
        vs[a] = X.v - X.by * t1;
        ws[a] = X.w - X.bz * t1;
        bys[a] = X.by * t2;
        bzs[a] = X.bz * t2;
    }
    // double-star states (shared by both sides)
    const double sg = bn >= 0.0 ? 1.0 : -1.0;
    const double irL = mrsqrt(ds[0]), irR = mrsqrt(ds[1]);
    const double rL = ds[0] * irL, rR = ds[1] * irR;
    const double isum = 1.0 / (rL + rR);
    const double vss = (rL * vs[0] + rR * vs[1] + sg * (bys[1] - bys[0])) * isum;
    const double wss = (rL * ws[0] + rR * ws[1] + sg * (bzs[1] - bzs[0])) * isum;
    const double byss = (rL * bys[1] + rR * bys[0] + sg * rL * rR * (vs[1] - vs[0])) * isum;
    const double bzss = (rL * bzs[1] + rR * bzs[0] + sg * rL * rR * (ws[1] - ws[0])) * isum;
    const double vbss = sM * bn + vss * byss + wss * bzss;

    // the side whose fan contains x/t = 0
    const bool left = sM >= 0.0;
    const W7 &X = left ? L : R;
    const int a = left ? 0 : 1;
    const double S = left ? sL : sR;
    const double pt = left ? ptL : ptR;
    const double e = left ? eL : eR;
    const double r = left ? rL : rR;
    const double car = fabs(bn) * (left ? irL : irR);
    const double ss = left ? sM - car : sM + car;
    const bool star_only = left ? (ss >= 0.0) : (ss <= 0.0);
    // its single-star energy and the double-star correction
    const double vbs = sM * bn + vs[a] * bys[a] + ws[a] * bzs[a];
    const double vbx = X.u * bn + X.v * X.by + X.w * X.bz;
    const double esa = ((S - X.u) * e - pt * X.u + pts * sM + bn * (vbx - vbs)) * issm[a];
    const double ess = left ? esa - r * sg * (vbs - vbss) : esa + r * sg * (vbs - vbss);
    const bool outer = left ? (sL > 0.0) : (sR < 0.0);
    const double cS = outer ? 0.0 : S;
    const double cSS = (outer || star_only) ? 0.0 : ss;

    const double vb = vbx;
    const double mu = X.d * X.u;
    // physical flux F(W) of the chosen side (Sec. 2.1, sweep frame)
    const double F0 = mu;
    const double F1 = mu * X.u + pt - bn2;
    const double F2 = mu * X.v - bn * X.by;
    const double F3 = mu * X.w - bn * X.bz;
    const double F4 = (e + pt) * X.u - bn * vb;
    const double F5 = X.by * X.u - bn * X.v;
    const double F6 = X.bz * X.u - bn * X.w;
    // U* - U and U** - U*
    const double dsa = ds[a];
    const double dU0 = dsa - X.d;
    const double dU1 = dsa * sM - mu;
    const double dU2 = dsa * vs[a] - X.d * X.v;
    const double dU3 = dsa * ws[a] - X.d * X.w;
    const double dU4 = esa - e;
    const double dU5 = bys[a] - X.by;
    const double dU6 = bzs[a] - X.bz;
    const double dV2 = dsa * (vss - vs[a]);
    const double dV3 = dsa * (wss - ws[a]);
    const double dV4 = ess - esa;
    const double dV5 = byss - bys[a];
    const double dV6 = bzss - bzs[a];
    f[0] = F0 + cS * dU0;
    f[1] = F1 + cS * dU1;
    f[2] = F2 + cS * dU2 + cSS * dV2;
    f[3] = F3 + cS * dU3 + cSS * dV3;
    f[4] = F4 + cS * dU4 + cSS * dV4;
    f[5] = F5 + cS * dU5 + cSS * dV5;
    f[6] = F6 + cS * dU6 + cSS * dV6;

    const double vtol = kUpwindTiny * (cmax + fabs(L.u) + fabs(R.u));
    const double ind = sM > vtol ? 1.0 : (sM < -vtol ? -1.0 : 0.0);
    upw = sL > 0.0 ? 1.0 : (sR < 0.0 ? -1.0 : ind);
}

// ---------------------------------------------------------------------------
// Characteristic eigen-system of the 1D primitive system (Sec. 2.2 Step 6,
// item 3) with the Roe-Balsara normalisation; left eigenvectors in closed
// form (they are the exact inverse of the right ones).
// Waves m = 0..6: u-cf, u-ca, u-cs, u, u+cs, u+ca, u+cf.
// ---------------------------------------------------------------------------
struct Eigen {
    double d, sqd, asq, a, ia2;   // rho, sqrt(rho), a^2 = gP/rho, a, 1/a^2
    double cf, cs, af, as;        // fast/slow speeds and alpha_f, alpha_s
    double by, bz, s;             // beta_t1, beta_t2, sign(B_n)
    // left-eigenvector coefficients
    double nf, ns, qf, qs, pf, ps, bf, bs, sr;
};

VLCT_DEV void eigen_setup(const W7 &c, double bn_in, double gam, Eigen &E)
{
    // field components below kBperpTiny of the magnetosonic scale
    // sqrt(gP + B^2) are rounding noise and are zero here, so noise cannot
    // turn the B_perp direction (compared in squares)
    const double gp = gam * c.p;
    const double tiny2 =
        kBperpTiny * kBperpTiny * (gp + bn_in * bn_in + c.by * c.by + c.bz * c.bz);
    const double bn = bn_in * bn_in <= tiny2 ? 0.0 : bn_in;
    const double bt1 = c.by * c.by <= tiny2 ? 0.0 : c.by;
    const double bt2 = c.bz * c.bz <= tiny2 ? 0.0 : c.bz;
    // r = 1/sqrt(rho), q = 1/sqrt(gP): every root and reciprocal of rho and gP
    // below follows from these two
    const double r = mrsqrt(c.d), q = mrsqrt(gp);
    const double id = r * r;
    E.d = c.d;
    E.sqd = c.d * r;
    E.asq = gp * id;
    E.a = gp * q * r;          // sqrt(gP / rho)
    E.ia2 = c.d * q * q;       // rho / (gP)
    const double bp2 = bt1 * bt1 + bt2 * bt2;
    const double t = gp - (bn * bn + bp2);
    const double disc = msqrt(t * t + 4.0 * gp * bp2);
    const double cf2 = (gp + bn * bn + bp2 + disc) * (0.5 * id);
    E.cf = msqrt(cf2);
    // c_s = a |B_n| / (sqrt(rho) c_f), the root of gP B_n^2 / (rho^2 c_f^2)
    E.cs = E.a * fabs(bn) * r / E.cf;
    const bool haveperp = bp2 > tiny2;
    const double ibp = mrsqrt(haveperp ? bp2 : 1.0);
    E.by = haveperp ? bt1 * ibp : 0.70710678118654752440;
    E.bz = haveperp ? bt2 * ibp : 0.70710678118654752440;
    const double tdiff = t;
    const bool split = disc > kCfCsTiny * c.d * cf2;
    const double idisc = 0.5 / disc;
    const double af2 = fmin(fmax((disc + tdiff) * idisc, 0.0), 1.0);
    const double as2 = fmin(fmax((disc - tdiff) * idisc, 0.0), 1.0);
    E.af = split ? msqrt(af2) : 1.0;
    E.as = split ? msqrt(as2) : 0.0;
    E.s = bn >= 0.0 ? 1.0 : -1.0;
    const double ia2 = E.ia2;
    E.nf = 0.5 * E.af * E.cf * ia2;
    E.ns = 0.5 * E.as * E.cs * ia2;
    E.qf = 0.5 * E.s * E.as * E.cs * ia2;
    E.qs = 0.5 * E.s * E.af * E.cf * ia2;
    E.pf = 0.5 * E.af * ia2 * id;
    E.ps = 0.5 * E.as * ia2 * id;
    E.bf = 0.5 * E.as * q;     // q = 1 / (a sqrt(rho))
    E.bs = -0.5 * E.af * q;
    E.sr = 0.5 * E.s * r;
}

// characteristic amplitudes a = L dW of a primitive increment dW
VLCT_DEV void project(const Eigen &E, const double dw[7], double a[7])
{
    const double vpar = E.by * dw[2] + E.bz * dw[3];
    const double vperp = -E.bz * dw[2] + E.by * dw[3];
    const double bpar = E.by * dw[5] + E.bz * dw[6];
    const double bperp = -E.bz * dw[5] + E.by * dw[6];
    const double hf = E.pf * dw[4] + E.bf * bpar;
    const double gf = E.nf * dw[1] - E.qf * vpar;
    const double hs = E.ps * dw[4] + E.bs * bpar;
    const double gs = E.ns * dw[1] + E.qs * vpar;
    a[0] = hf - gf;
    a[6] = hf + gf;
    a[2] = hs - gs;
    a[4] = hs + gs;
    a[1] = 0.5 * vperp + E.sr * bperp;
    a[5] = 0.5 * vperp - E.sr * bperp;
    a[3] = dw[0] - dw[4] * E.ia2;
}

// primitive increment dW = R a of characteristic amplitudes a
VLCT_DEV void unproject(const Eigen &E, const double a[7], double dw[7])
{
    const double fsum = a[0] + a[6], fdif = a[6] - a[0];
    const double ssum = a[2] + a[4], sdif = a[4] - a[2];
    const double asum = a[1] + a[5], adif = a[5] - a[1];
    const double tpar = -E.s * (E.as * E.cs * fdif - E.af * E.cf * sdif);
    const double bmag = E.a * E.sqd * (E.as * fsum - E.af * ssum);
    const double sb = E.s * E.sqd * adif;
    dw[0] = E.d * (E.af * fsum + E.as * ssum) + a[3];
    dw[1] = E.af * E.cf * fdif + E.as * E.cs * sdif;
    dw[2] = E.by * tpar - E.bz * asum;
    dw[3] = E.bz * tpar + E.by * asum;
    dw[4] = E.d * E.asq * (E.af * fsum + E.as * ssum);
    dw[5] = E.by * bmag + E.bz * sb;
    dw[6] = E.bz * bmag - E.by * sb;
}

VLCT_DEV void to_arr(const W7 &w, double x[7])
{
    x[0] = w.d; x[1] = w.u; x[2] = w.v; x[3] = w.w; x[4] = w.p; x[5] = w.by; x[6] = w.bz;
}

VLCT_DEV W7 from_arr(const double x[7])
{
    return W7{x[0], x[1], x[2], x[3], x[4], x[5], x[6]};
}

// floor an interface state; returns status bits
VLCT_DEV uint32_t floor_state(W7 &w)
{
    uint32_t st = 0;
    if (!(w.d >= kFloorRho)) { w.d = kFloorRho; st |= kStatusDensityFloor; }
    if (!(w.p >= kFloorP)) { w.p = kFloorP; st |= kStatusPressureFloor; }
    return st;
}

// ---------------------------------------------------------------------------
// PLMC (Sec. 2.2 Step 6 items 1-6, Eq. limiter): left/right/centred/van Leer
// primitive differences projected with the eigenvectors of the cell,
// limited, projected back; fm = state at the low face, fp = at the high face.
// ---------------------------------------------------------------------------
template <bool CHAR>
VLCT_DEV void plmc(const W7 &wm, const W7 &w0, const W7 &wp, double bn,
                                     double gam, W7 &fm, W7 &fp)
{
    // CHAR = false is PLMP: the same steps with the projections skipped
    double xm[7], x0[7], xp[7];
    to_arr(wm, xm);
    to_arr(w0, x0);
    to_arr(wp, xp);
    double dl[7], dr[7], dc[7], dv[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        dl[c] = x0[c] - xm[c];
        dr[c] = xp[c] - x0[c];
        dc[c] = 0.5 * (xp[c] - xm[c]);
        const double pr = dl[c] * dr[c];
        dv[c] = pr > 0.0 ? 2.0 * pr / (dl[c] + dr[c]) : 0.0;
    }
    Eigen E;
    double al[7], ar[7], ac[7], av[7], am[7];
    if (CHAR) {
        eigen_setup(w0, bn, gam, E);
        project(E, dl, al);
        project(E, dr, ar);
        project(E, dc, ac);
        project(E, dv, av);
    } else {
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            al[c] = dl[c];
            ar[c] = dr[c];
            ac[c] = dc[c];
            av[c] = dv[c];
        }
    }
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        const double lim = fmin(fmin(2.0 * fabs(al[m]), 2.0 * fabs(ar[m])),
                                fmin(fabs(ac[m]), fabs(av[m])));
        am[m] = al[m] * ar[m] > 0.0 ? copysign(lim, ac[m]) : 0.0;
    }
    double dw[7];
    if (CHAR) {
        unproject(E, am, dw);
    } else {
#pragma unroll
        for (int c = 0; c < 7; ++c) dw[c] = am[c];
    }
    double p[7], q[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        p[c] = x0[c] + 0.5 * dw[c];
        q[c] = x0[c] - 0.5 * dw[c];
    }
    fp = from_arr(p);
    fm = from_arr(q);
}

// ---------------------------------------------------------------------------
// PPMC (third order, limited in characteristic variables).  The paper defers
// to Felker & Stone (2018) without formulas; this implements the reading used
// throughout the library: stencil differences relative to the cell (rounding-
// level differences set to zero), fourth-order face values, Colella-Sekora
// face limiter, extremum-preserving parabola limiter / overshoot correction
// per characteristic field, back projection, then each face primitive clamped
// between the two cells that share the face.
// ---------------------------------------------------------------------------
VLCT_DEV double ppm_face(double am, double a0, double ap, double app)
{
    double f = (7.0 / 12.0) * (a0 + ap) - (1.0 / 12.0) * (am + app);
    if ((f - a0) * (ap - f) < 0.0) {
        const double d2 = 3.0 * (a0 - 2.0 * f + ap);
        const double d2l = am - 2.0 * a0 + ap;
        const double d2r = a0 - 2.0 * ap + app;
        double lim = 0.0;
        if (d2 * d2l > 0.0 && d2 * d2r > 0.0)
            lim = copysign(fmin(fmin(kPpmC * fabs(d2l), kPpmC * fabs(d2r)), fabs(d2)), d2);
        // all three curvature estimates are h^2 f'' on a parabola: with
        // lim = d2 (limiter not binding) this gives back the fourth-order f
        f = 0.5 * (a0 + ap) - lim * (1.0 / 6.0);
    }
    return f;
}

template <bool CHAR>
VLCT_DEV void ppmc(const W7 &wmm, const W7 &wm, const W7 &w0, const W7 &wp,
                                     const W7 &wpp, double bn, double gam, W7 &fm, W7 &fp)
{
    // CHAR = false is PPMP: the same steps with the projections skipped
    // stencil differences relative to the cell; a difference within kPpmTie of
    // the magnitudes it is taken from counts as zero, so that rounding noise at
    // a symmetric extremum cannot pick the other branch of the extremum test
    Eigen E;
    double fv, fb;
    if (CHAR) {
        eigen_setup(w0, bn, gam, E);
        fv = E.cf;
        fb = E.sqd * E.cf;
    } else {
        fv = fast_speed(w0.d, w0.p, bn, w0.by, w0.bz, gam);
        fb = msqrt(w0.d) * fv;
    }
    // magnitude floors of the tie test: c_f for velocities, sqrt(rho) c_f for B
    const double floor_c[7] = {0.0, fv, fv, fv, 0.0, fb, fb};
    double x0[7], xs[4][7];
    to_arr(w0, x0);
    {
        const W7 *nb[4] = {&wmm, &wm, &wp, &wpp};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double t[7];
            to_arr(*nb[q], t);
#pragma unroll
            for (int c = 0; c < 7; ++c) {
                const double d = t[c] - x0[c];
                xs[q][c] = fabs(d) <= kPpmTie * (fabs(t[c]) + fabs(x0[c]) + floor_c[c]) ? 0.0 : d;
            }
        }
    }
    double a[4][7];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (CHAR) {
            project(E, xs[s], a[s]);
        } else {
#pragma unroll
            for (int c = 0; c < 7; ++c) a[s][c] = xs[s][c];
        }
    }
    double dplus[7], dminus[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        // characteristic values relative to the cell (a0 = 0)
        const double a_2 = a[0][m], a_1 = a[1][m], a1 = a[2][m], a2 = a[3][m];
        const double a0 = 0.0;
        const double fl = ppm_face(a_2, a_1, a0, a1);
        const double fr = ppm_face(a_1, a0, a1, a2);
        double dp = fr - a0, dm = a0 - fl;
        if (dp * dm <= 0.0 || (a1 - a0) * (a0 - a_1) <= 0.0) {
            const double d2 = 6.0 * (fl - 2.0 * a0 + fr);
            const double d2c = a_1 - 2.0 * a0 + a1;
            const double d2l = a_2 - 2.0 * a_1 + a0;
            const double d2r = a0 - 2.0 * a1 + a2;
            double lim = 0.0;
            if (d2 * d2c > 0.0 && d2 * d2l > 0.0 && d2 * d2r > 0.0)
                lim = copysign(fmin(fmin(kPpmC * fabs(d2l), kPpmC * fabs(d2r)),
                                    fmin(kPpmC * fabs(d2c), fabs(d2))), d2);
            const double ratio = d2 != 0.0 ? lim / d2 : 0.0;
            dp = dp * ratio;
            dm = dm * ratio;
        } else {
            if (fabs(dp) >= 2.0 * fabs(dm)) dp = 2.0 * dm;
            if (fabs(dm) >= 2.0 * fabs(dp)) dm = 2.0 * dp;
        }
        // the limited interface values stay between the cell's (0) and the
        // neighbour's characteristic values
        dplus[m] = fmax(fmin(0.0, a1), fmin(dp, fmax(0.0, a1)));
        dminus[m] = fmax(fmin(0.0, a_1), fmin(-dm, fmax(0.0, a_1)));
    }
    double wpl[7], wmi[7];
    if (CHAR) {
        unproject(E, dplus, wpl);
        unproject(E, dminus, wmi);
    } else {
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            wpl[c] = dplus[c];
            wmi[c] = dminus[c];
        }
    }
    double xl[7], xr[7], p[7], q[7];
    to_arr(wm, xl);
    to_arr(wp, xr);
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        const double up = x0[c] + wpl[c];
        const double um = x0[c] + wmi[c];
        // bound between the neighbouring cell values
        double vp = fmax(fmin(x0[c], xr[c]), fmin(up, fmax(x0[c], xr[c])));
        double vm = fmax(fmin(x0[c], xl[c]), fmin(um, fmax(x0[c], xl[c])));
        // a bound that acted beyond rounding: Colella-Woodward monotonicity
        // constraints on this primitive's interface pair
        const double tol = kPpmTie * (fabs(x0[c]) + fabs(xl[c]) + fabs(xr[c]) + floor_c[c]);
        if (fabs(vp - up) > tol || fabs(vm - um) > tol) {
            const double dpp = vp - x0[c], dmm = x0[c] - vm;
            if (dpp * dmm <= 0.0) {
                vp = x0[c];
                vm = x0[c];
            } else {
                if (fabs(dpp) >= 2.0 * fabs(dmm)) vp = x0[c] + 2.0 * dmm;
                if (fabs(dmm) >= 2.0 * fabs(dpp)) vm = x0[c] - 2.0 * dpp;
            }
        }
        p[c] = vp;
        q[c] = vm;
    }
    fp = from_arr(p);
    fm = from_arr(q);
}

}  // namespace vlct
