/*
 * vlct_ref.c -- CPU oracle for one Van Leer + Constrained Transport (VL+CT)
 * time step of 3D ideal MHD, written from Caddy & Schneider, "Cholla-MHD"
 * (Sec. 2.1 equations, Sec. 2.2 Steps 1-10).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain FP64 C compiled with -ffp-contract=off.
 * It shares no code with the GPU library; only the tests, the smoke entry
 * point and the benchmark's CPU-baseline leg may load it.
 *
 * Structure: every stage is computed over the whole (ghost-padded) grid into
 * full arrays -- cell primitives, reconstructed interface states, face fluxes,
 * edge EMFs -- and then the interior cells and faces are updated.  Nothing is
 * blocked, fused or reordered.
 *
 * Readings of points the paper leaves open (each is documented with the
 * design notes of the repository):
 *  - the half-step update (Step 5) uses dt/2, since Step 5 advances to
 *    t + dt/2; flux differences are F(j+1/2)-F(j-1/2) in every direction;
 *  - Step 8 repeats the edge-EMF computation of Step 4 with the corrector
 *    fluxes and the half-step cell state as reference field;
 *  - edge EMF (Eq. emf-edge): all four slope terms are (face EMF - cell
 *    reference EMF) of the upwind cell, each with weight 1/4; the upwind
 *    direction is the sign of the interface velocity of the adjacent face's
 *    HLLD solution (S_M, whose sign is that of the mass flux rho* S_M), and a
 *    velocity within 1e-12 of the local signal speed counts as zero and takes
 *    the average (Eq. emf-upwind-slope);
 *  - the CFL step (Eq. dt) uses, per direction l, the fast speed with B_l as
 *    the longitudinal field and is evaluated as C / max((|v_l|+c_f,l)/d_l);
 *  - HLLD follows Miyoshi & Kusano (2005): min/max wave-speed estimate,
 *    degenerate star states when |rho(S-u)(S-S_M) - Bn^2| < 1e-8 p_T*;
 *  - characteristic eigenvectors use the Roe-Balsara normalisation with
 *    beta = 1/sqrt(2) when B_perp vanishes and alpha_f = 1 when c_f = c_s;
 *    field components below 1e-12 sqrt(gP + B^2) count as zero there;
 *  - boundaries: every stage's state is extended by index mapping (wrap on
 *    periodic axes, clamp on outflow axes; face fields clamp their normal
 *    index into [0, n] and their transverse indices into [0, n-1]);
 *  - floors: rho and P derived from a conserved state, and reconstructed
 *    interface states, are floored at 1e-20 (the conserved state is never
 *    modified); each floor sets a status bit;
 *  - PLMP / PPMP: the same reconstructions with the projections skipped
 *    (limiting in the primitive variables, Step 6's closing remark);
 *  - PPMC: characteristic projection of the stencil differences (rounding-
 *    level primitive differences, below 1e-12 of the values' magnitude with
 *    c_f and sqrt(rho) c_f as floors for velocity and field, taken as zero),
 *    4th-order interface values, Colella-Sekora interface and
 *    extremum-preserving limiters, then interface primitives clamped between
 *    the neighbouring cell values.
 */
#include "vlct_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NG 4                /* ghost layers of the padded working grid */
#define FLOOR_RHO 1.0e-20
#define FLOOR_P 1.0e-20
#define HLLD_DEGEN 1.0e-8   /* degenerate-star threshold relative to p_T* */
#define BPERP_TINY 1.0e-12  /* B_n, B_perp below this * sqrt(gP+B^2): zero / beta = 1/sqrt2 */
#define CFCS_TINY 1.0e-12   /* c_f^2 - c_s^2 below this * c_f^2 => alpha_f = 1 */
#define PPM_C 1.25          /* Colella-Sekora curvature-ratio constant */
#define UPWIND_TINY 1.0e-12 /* |S_M| below this * signal speed counts as zero */
#define PPM_TIE 1.0e-12     /* PPMC: relative size of a stencil difference taken as zero */

/* ------------------------------------------------------------------------- */
/* Primitive-variable physics of one state (Sec. 2.1)                         */
/* ------------------------------------------------------------------------- */

/* Fast and slow magnetosonic speeds (Sec. 2.2 Step 1, c_{f,s} equation),
 * bn = field component along the direction of propagation.  The discriminant
 * (gP + B^2)^2 - 4 gP bn^2 is evaluated in the algebraically identical form
 * (gP - B^2)^2 + 4 gP B_perp^2, which cannot cancel, and c_s^2 as the product
 * of the roots divided by c_f^2 (c_f^2 c_s^2 = gP bn^2 / rho^2). */
static void speeds_sq(double rho, double p, double bn, double bt1, double bt2, double gamma,
                      double *cf2, double *cs2, double *disc_out)
{
    double gp = gamma * p;
    double bperp2 = bt1 * bt1 + bt2 * bt2;
    double b2 = bn * bn + bperp2;
    double t = gp - b2;
    double disc = sqrt(t * t + 4.0 * gp * bperp2);
    double f2 = (gp + b2 + disc) / (2.0 * rho);
    *cf2 = f2;
    *cs2 = f2 > 0.0 ? (gp * bn * bn) / (rho * rho * f2) : 0.0;
    if (disc_out) *disc_out = disc;
}

void vref_wave_speeds(double rho, double p, double bn, double bt1, double bt2,
                      double gamma, double *cf, double *cs)
{
    double f2, s2;
    speeds_sq(rho, p, bn, bt1, bt2, gamma, &f2, &s2, NULL);
    *cf = sqrt(f2);
    *cs = sqrt(s2);
}

static double fast_speed(double rho, double p, double bn, double bt1, double bt2,
                         double gamma)
{
    double cf, cs;
    vref_wave_speeds(rho, p, bn, bt1, bt2, gamma, &cf, &cs);
    return cf;
}

/* Physical flux F_x of Sec. 2.1 written in the sweep frame (n, t1, t2). */
void vref_phys_flux(const double w[7], double bn, double gamma, double f[7])
{
    double rho = w[0], u = w[1], v = w[2], ww = w[3], p = w[4], by = w[5], bz = w[6];
    double b2 = bn * bn + by * by + bz * bz;
    double pt = p + 0.5 * b2;
    double en = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + ww * ww) + 0.5 * b2;
    double vb = u * bn + v * by + ww * bz;
    f[0] = rho * u;
    f[1] = rho * u * u + pt - bn * bn;
    f[2] = rho * u * v - bn * by;
    f[3] = rho * u * ww - bn * bz;
    f[4] = (en + pt) * u - bn * vb;
    f[5] = by * u - bn * v;
    f[6] = bz * u - bn * ww;
}

static void prim_to_cons(const double w[7], double bn, double gamma, double U[7])
{
    double rho = w[0], u = w[1], v = w[2], ww = w[3], p = w[4], by = w[5], bz = w[6];
    U[0] = rho;
    U[1] = rho * u;
    U[2] = rho * v;
    U[3] = rho * ww;
    U[4] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + ww * ww)
           + 0.5 * (bn * bn + by * by + bz * bz);
    U[5] = by;
    U[6] = bz;
}

/* ------------------------------------------------------------------------- */
/* HLLD Riemann solver (Sec. 2.2 Step 3; Miyoshi & Kusano 2005)               */
/* ------------------------------------------------------------------------- */

typedef struct {
    double U[7];     /* conserved state */
    double F[7];     /* physical flux */
    double u, pt;    /* normal velocity, total pressure */
    double vb;       /* v . B */
} hlld_side;

static void hlld_side_init(const double w[7], double bn, double gamma, hlld_side *s)
{
    prim_to_cons(w, bn, gamma, s->U);
    vref_phys_flux(w, bn, gamma, s->F);
    s->u = w[1];
    s->pt = w[4] + 0.5 * (bn * bn + w[5] * w[5] + w[6] * w[6]);
    s->vb = w[1] * bn + w[2] * w[5] + w[3] * w[6];
}

void vref_hlld(const double wl[7], const double wr[7], double bn, double gamma,
               double flux[8])
{
    hlld_side L, R;
    hlld_side_init(wl, bn, gamma, &L);
    hlld_side_init(wr, bn, gamma, &R);

    /* outer wave speeds: min/max estimate (M&K 2005, eq. 67) */
    double cfl = fast_speed(wl[0], wl[4], bn, wl[5], wl[6], gamma);
    double cfr = fast_speed(wr[0], wr[4], bn, wr[5], wr[6], gamma);
    double cmax = cfl > cfr ? cfl : cfr;
    double sl = (wl[1] < wr[1] ? wl[1] : wr[1]) - cmax;
    double sr = (wl[1] > wr[1] ? wl[1] : wr[1]) + cmax;

    if (sl > 0.0) { memcpy(flux, L.F, sizeof(L.F)); flux[7] = 1.0; return; }
    if (sr < 0.0) { memcpy(flux, R.F, sizeof(R.F)); flux[7] = -1.0; return; }

    /* contact speed and star total pressure (M&K eqs. 38, 41) */
    double ql = (sl - wl[1]) * wl[0];
    double qr = (sr - wr[1]) * wr[0];
    double sm = (qr * wr[1] - ql * wl[1] - R.pt + L.pt) / (qr - ql);
    double pts = (qr * L.pt - ql * R.pt + ql * qr * (wr[1] - wl[1])) / (qr - ql);

    /* upwind indicator for the CT slopes (Eq. emf-upwind-slope): the sign of
     * the interface velocity S_M (the sign of the mass flux rho* S_M), zero
     * when |S_M| is within UPWIND_TINY of the local signal speed */
    double vtol = UPWIND_TINY * (cmax + fabs(wl[1]) + fabs(wr[1]));
    flux[7] = sm > vtol ? 1.0 : (sm < -vtol ? -1.0 : 0.0);

    /* single-star states (M&K eqs. 43-48) */
    const double *wa[2] = {wl, wr};
    const hlld_side *sa[2] = {&L, &R};
    double S[2] = {sl, sr};
    double Us[2][7], rhos[2], vs[2], ws[2], bys[2], bzs[2], vbs[2];
    for (int a = 0; a < 2; ++a) {
        const double *w = wa[a];
        double su = S[a] - w[1];
        double ssm = S[a] - sm;
        rhos[a] = w[0] * su / ssm;
        double d = w[0] * su * ssm - bn * bn;
        if (fabs(d) < HLLD_DEGEN * pts) {
            vs[a] = w[2];
            ws[a] = w[3];
            bys[a] = w[5];
            bzs[a] = w[6];
        } else {
            double t = bn * (sm - w[1]) / d;
            vs[a] = w[2] - w[5] * t;
            ws[a] = w[3] - w[6] * t;
            double t2 = (w[0] * su * su - bn * bn) / d;
            bys[a] = w[5] * t2;
            bzs[a] = w[6] * t2;
        }
        vbs[a] = sm * bn + vs[a] * bys[a] + ws[a] * bzs[a];
        double es = (su * sa[a]->U[4] - sa[a]->pt * w[1] + pts * sm
                     + bn * (sa[a]->vb - vbs[a])) / ssm;
        Us[a][0] = rhos[a];
        Us[a][1] = rhos[a] * sm;
        Us[a][2] = rhos[a] * vs[a];
        Us[a][3] = rhos[a] * ws[a];
        Us[a][4] = es;
        Us[a][5] = bys[a];
        Us[a][6] = bzs[a];
    }

    /* double-star states (M&K eqs. 49-63) */
    double sgn = bn >= 0.0 ? 1.0 : -1.0;
    double rl = sqrt(rhos[0]), rr = sqrt(rhos[1]);
    double ssl = sm - fabs(bn) / rl;
    double ssr = sm + fabs(bn) / rr;
    double inv = 1.0 / (rl + rr);
    double vss = (rl * vs[0] + rr * vs[1] + sgn * (bys[1] - bys[0])) * inv;
    double wss = (rl * ws[0] + rr * ws[1] + sgn * (bzs[1] - bzs[0])) * inv;
    double byss = (rl * bys[1] + rr * bys[0] + sgn * rl * rr * (vs[1] - vs[0])) * inv;
    double bzss = (rl * bzs[1] + rr * bzs[0] + sgn * rl * rr * (ws[1] - ws[0])) * inv;
    double vbss = sm * bn + vss * byss + wss * bzss;
    double Uss[2][7];
    for (int a = 0; a < 2; ++a) {
        Uss[a][0] = rhos[a];
        Uss[a][1] = rhos[a] * sm;
        Uss[a][2] = rhos[a] * vss;
        Uss[a][3] = rhos[a] * wss;
        Uss[a][5] = byss;
        Uss[a][6] = bzss;
    }
    Uss[0][4] = Us[0][4] - rl * sgn * (vbs[0] - vbss);
    Uss[1][4] = Us[1][4] + rr * sgn * (vbs[1] - vbss);

    /* flux of the region containing x/t = 0 (M&K eqs. 64-66) */
    int a;
    double ss;
    if (sm >= 0.0) { a = 0; ss = ssl; } else { a = 1; ss = ssr; }
    const hlld_side *s = sa[a];
    int in_star_only = (a == 0) ? (ssl >= 0.0) : (ssr <= 0.0);
    for (int c = 0; c < 7; ++c) {
        double fs = s->F[c] + S[a] * (Us[a][c] - s->U[c]);
        if (in_star_only)
            flux[c] = fs;
        else
            flux[c] = fs + ss * (Uss[a][c] - Us[a][c]);
    }
}

/* ------------------------------------------------------------------------- */
/* Characteristic eigen-system of the 1D primitive MHD equations             */
/* (Sec. 2.2 Step 6 item 3: eigenvectors of the Athena appendix, Roe-Balsara  */
/* normalisation), w = (rho, u, v, w, P, B_t1, B_t2), normal field bn.        */
/* ------------------------------------------------------------------------- */

void vref_eigen(const double w[7], double bn, double gamma, double R[49], double L[49],
                double lam[7])
{
    double rho = w[0], u = w[1], p = w[4], by = w[5], bz = w[6];
    /* field components below 1e-12 of the magnetosonic scale sqrt(gP + B^2)
     * are rounding noise: each such component (B_n, B_t1, B_t2) is zero, so
     * that noise cannot turn the B_perp direction and with it a projection
     * that is exactly zero into a tiny one of either sign; a B_perp below it
     * takes the degenerate-direction convention */
    double bscale = sqrt(gamma * p + bn * bn + by * by + bz * bz);
    if (fabs(bn) <= BPERP_TINY * bscale) bn = 0.0;
    if (fabs(by) <= BPERP_TINY * bscale) by = 0.0;
    if (fabs(bz) <= BPERP_TINY * bscale) bz = 0.0;
    double a2 = gamma * p / rho;
    double a = sqrt(a2);
    double cf, cs;
    vref_wave_speeds(rho, p, bn, by, bz, gamma, &cf, &cs);
    double ca = fabs(bn) / sqrt(rho);
    double sqr = sqrt(rho);

    double bperp = sqrt(by * by + bz * bz);
    double bety, betz;
    if (bperp > BPERP_TINY * bscale) {
        bety = by / bperp;
        betz = bz / bperp;
    } else {
        bety = betz = 1.0 / sqrt(2.0);
    }
    /* Roe-Balsara weights: alpha_f^2 = (a^2 - c_s^2)/(c_f^2 - c_s^2) and
     * alpha_s^2 = (c_f^2 - a^2)/(c_f^2 - c_s^2), written with the
     * discriminant d = rho (c_f^2 - c_s^2) as (d +- (gP - B^2)) / (2 d) so that
     * they are exact 0/1 where B_perp = 0. */
    double cf2, cs2, disc;
    speeds_sq(rho, p, bn, by, bz, gamma, &cf2, &cs2, &disc);
    double af, as;
    double tdiff = gamma * p - (bn * bn + by * by + bz * bz);
    if (disc > CFCS_TINY * rho * cf2) {
        double af2 = (disc + tdiff) / (2.0 * disc);
        double as2 = (disc - tdiff) / (2.0 * disc);
        if (af2 < 0.0) af2 = 0.0;
        if (af2 > 1.0) af2 = 1.0;
        if (as2 < 0.0) as2 = 0.0;
        if (as2 > 1.0) as2 = 1.0;
        af = sqrt(af2);
        as = sqrt(as2);
    } else {
        af = 1.0;
        as = 0.0;
    }
    double s = bn >= 0.0 ? 1.0 : -1.0;

    double col[7][7]; /* col[m] = right eigenvector of wave m */
    for (int m = 0; m < 7; ++m)
        for (int r = 0; r < 7; ++r) col[m][r] = 0.0;
    for (int e = -1; e <= 1; e += 2) {
        /* fast waves (m = 0: u - cf, m = 6: u + cf) */
        double *f = col[e < 0 ? 0 : 6];
        f[0] = rho * af;
        f[1] = e * af * cf;
        f[2] = -e * s * as * cs * bety;
        f[3] = -e * s * as * cs * betz;
        f[4] = rho * af * a2;
        f[5] = as * a * sqr * bety;
        f[6] = as * a * sqr * betz;
        /* slow waves (m = 2: u - cs, m = 4: u + cs) */
        double *sl = col[e < 0 ? 2 : 4];
        sl[0] = rho * as;
        sl[1] = e * as * cs;
        sl[2] = e * s * af * cf * bety;
        sl[3] = e * s * af * cf * betz;
        sl[4] = rho * as * a2;
        sl[5] = -af * a * sqr * bety;
        sl[6] = -af * a * sqr * betz;
        /* Alfven waves (m = 1: u - ca, m = 5: u + ca) */
        double *al = col[e < 0 ? 1 : 5];
        al[2] = -betz;
        al[3] = bety;
        al[5] = e * s * sqr * betz;
        al[6] = -e * s * sqr * bety;
    }
    col[3][0] = 1.0; /* entropy wave */

    for (int r = 0; r < 7; ++r)
        for (int m = 0; m < 7; ++m) R[r * 7 + m] = col[m][r];

    /* Left eigenvectors (rows of L = R^{-1}) in closed form.  The fast/slow
     * pairs split into a part acting on (rho, P, B along beta) and a part on
     * (u, v along beta); using c_f^2 alpha_f^2 + c_s^2 alpha_s^2 = a^2 the
     * inverse has the coefficients below.  Written out (rather than inverted
     * numerically) so that entries that vanish exactly -- e.g. the coupling
     * of the Alfven and entropy waves to u -- are exact zeros. */
    double ia2 = 1.0 / a2;
    double nf = 0.5 * af * cf * ia2, ns = 0.5 * as * cs * ia2;
    double qf = 0.5 * s * as * cs * ia2, qs = 0.5 * s * af * cf * ia2;
    double pf = 0.5 * af * ia2 / rho, ps = 0.5 * as * ia2 / rho;
    double bf = 0.5 * as / (a * sqr), bs = -0.5 * af / (a * sqr);
    double sr = 0.5 * s / sqr;
    const double rows[7][7] = {
        {0.0, -nf, qf * bety, qf * betz, pf, bf * bety, bf * betz},      /* u - c_f */
        {0.0, 0.0, -0.5 * betz, 0.5 * bety, 0.0, -sr * betz, sr * bety}, /* u - c_a */
        {0.0, -ns, -qs * bety, -qs * betz, ps, bs * bety, bs * betz},    /* u - c_s */
        {1.0, 0.0, 0.0, 0.0, -ia2, 0.0, 0.0},                            /* u       */
        {0.0, ns, qs * bety, qs * betz, ps, bs * bety, bs * betz},       /* u + c_s */
        {0.0, 0.0, -0.5 * betz, 0.5 * bety, 0.0, sr * betz, -sr * bety}, /* u + c_a */
        {0.0, nf, -qf * bety, -qf * betz, pf, bf * bety, bf * betz},     /* u + c_f */
    };
    for (int r = 0; r < 7; ++r)
        for (int c = 0; c < 7; ++c) L[r * 7 + c] = rows[r][c];
    lam[0] = u - cf;
    lam[1] = u - ca;
    lam[2] = u - cs;
    lam[3] = u;
    lam[4] = u + cs;
    lam[5] = u + ca;
    lam[6] = u + cf;
}

static void matvec7(const double M[49], const double x[7], double y[7])
{
    for (int r = 0; r < 7; ++r) {
        double acc = 0.0;
        for (int c = 0; c < 7; ++c) acc += M[r * 7 + c] * x[c];
        y[r] = acc;
    }
}

static double sgn_pos(double x) { return x >= 0.0 ? 1.0 : -1.0; }
static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }

/* ------------------------------------------------------------------------- */
/* PLMC: piecewise-linear reconstruction limited in characteristic variables  */
/* (Sec. 2.2 Step 6, items 1-6 and Eq. limiter).  w[0..6] = cell i-1,         */
/* w[7..13] = cell i, w[14..20] = cell i+1.                                    */
/* ------------------------------------------------------------------------- */
void vref_plmc(const double w[21], double bn, double gamma, double face_minus[7],
               double face_plus[7])
{
    const double *wm = w, *w0 = w + 7, *wp = w + 14;
    double dL[7], dR[7], dC[7], dV[7];
    for (int c = 0; c < 7; ++c) {
        dL[c] = w0[c] - wm[c];
        dR[c] = wp[c] - w0[c];
        dC[c] = 0.5 * (wp[c] - wm[c]);
        dV[c] = (dL[c] * dR[c] > 0.0) ? 2.0 * dL[c] * dR[c] / (dL[c] + dR[c]) : 0.0;
    }
    double R[49], L[49], lam[7];
    vref_eigen(w0, bn, gamma, R, L, lam);
    double aL[7], aR[7], aC[7], aV[7], am[7];
    matvec7(L, dL, aL);
    matvec7(L, dR, aR);
    matvec7(L, dC, aC);
    matvec7(L, dV, aV);
    for (int m = 0; m < 7; ++m) {
        if (aL[m] * aR[m] > 0.0) {
            double lim = dmin(dmin(2.0 * fabs(aL[m]), 2.0 * fabs(aR[m])),
                              dmin(fabs(aC[m]), fabs(aV[m])));
            am[m] = sgn_pos(aC[m]) * lim;
        } else {
            am[m] = 0.0;
        }
    }
    double dw[7];
    matvec7(R, am, dw);
    for (int c = 0; c < 7; ++c) {
        face_plus[c] = w0[c] + 0.5 * dw[c];
        face_minus[c] = w0[c] - 0.5 * dw[c];
    }
}

/* PLMP: the same steps with the limiter applied to the primitive slopes, i.e.
 * skipping the projections of items 3 and 5 (Sec. 2.2 Step 6, closing remark). */
void vref_plmp(const double w[21], double face_minus[7], double face_plus[7])
{
    const double *wm = w, *w0 = w + 7, *wp = w + 14;
    for (int c = 0; c < 7; ++c) {
        double dL = w0[c] - wm[c], dR = wp[c] - w0[c], dC = 0.5 * (wp[c] - wm[c]);
        double dV = (dL * dR > 0.0) ? 2.0 * dL * dR / (dL + dR) : 0.0;
        double dm = 0.0;
        if (dL * dR > 0.0)
            dm = sgn_pos(dC) * dmin(dmin(2.0 * fabs(dL), 2.0 * fabs(dR)), dmin(fabs(dC), fabs(dV)));
        face_plus[c] = w0[c] + 0.5 * dm;
        face_minus[c] = w0[c] - 0.5 * dm;
    }
}

/* ------------------------------------------------------------------------- */
/* PPMC: piecewise-parabolic reconstruction in characteristic variables.     */
/* The paper gives no formulas (Sec. 2.2 Step 6 defers to Felker & Stone     */
/* 2018); this follows the reading stated in the header.                     */
/* w[0..34] = cells i-2 .. i+2.                                               */
/* ------------------------------------------------------------------------- */
static double ppm_face(double am, double a0, double ap, double app)
{
    /* face value between a0 and ap; neighbours am (left of a0), app (right of ap) */
    double f = (7.0 / 12.0) * (a0 + ap) - (1.0 / 12.0) * (am + app);
    if ((f - a0) * (ap - f) < 0.0) {
        double d2 = 3.0 * (a0 - 2.0 * f + ap);
        double d2l = am - 2.0 * a0 + ap;
        double d2r = a0 - 2.0 * ap + app;
        double lim = 0.0;
        if (d2 * d2l > 0.0 && d2 * d2r > 0.0) {
            double s = sgn_pos(d2);
            lim = s * dmin(dmin(PPM_C * fabs(d2l), PPM_C * fabs(d2r)), fabs(d2));
        }
        /* d2, d2l and d2r all equal h^2 f'' on a parabola, so the limited
         * value is written with d2 / 6: where the limiter does not bind
         * (lim = d2) it returns the fourth-order value f unchanged */
        f = 0.5 * (a0 + ap) - lim / 6.0;
    }
    return f;
}

static void ppm_basis(const double w[35], double bn, double gamma, int characteristic,
                      double face_minus[7], double face_plus[7]);

void vref_ppmc(const double w[35], double bn, double gamma, double face_minus[7],
               double face_plus[7])
{
    ppm_basis(w, bn, gamma, 1, face_minus, face_plus);
}

/* PPMP: PPM limited in the primitive variables (projections skipped). */
void vref_ppmp(const double w[35], double bn, double gamma, double face_minus[7],
               double face_plus[7])
{
    ppm_basis(w, bn, gamma, 0, face_minus, face_plus);
}

static void ppm_basis(const double w[35], double bn, double gamma, int characteristic,
                      double face_minus[7], double face_plus[7])
{
    const double *w0 = w + 14;
    double R[49], L[49], lam[7];
    if (characteristic) {
        vref_eigen(w0, bn, gamma, R, L, lam);
    } else {
        for (int q = 0; q < 49; ++q) R[q] = L[q] = (q % 8 == 0) ? 1.0 : 0.0;
    }
    /* characteristic values relative to the cell (the PPM steps only use
     * differences); a primitive difference within PPM_TIE of the magnitudes
     * it is taken from counts as zero, so rounding noise at a symmetric
     * extremum cannot select the other branch of the extremum test */
    /* magnitude floors of the tie test: velocities are measured against the
     * fast speed of the cell, field components against sqrt(rho) c_f */
    double cf0, cs0;
    vref_wave_speeds(w0[0], w0[4], bn, w0[5], w0[6], gamma, &cf0, &cs0);
    double floor_c[7] = {0.0, cf0, cf0, cf0, 0.0, sqrt(w0[0]) * cf0, sqrt(w0[0]) * cf0};
    double a[5][7];
    for (int s = 0; s < 5; ++s) {
        double dw[7];
        for (int c = 0; c < 7; ++c) {
            double d = w[7 * s + c] - w0[c];
            if (fabs(d) <= PPM_TIE * (fabs(w[7 * s + c]) + fabs(w0[c]) + floor_c[c])) d = 0.0;
            dw[c] = d;
        }
        matvec7(L, dw, a[s]);
    }
    double dminus[7], dplus[7];
    for (int m = 0; m < 7; ++m) {
        double a_2 = a[0][m], a_1 = a[1][m], a0 = a[2][m], a1 = a[3][m], a2 = a[4][m];
        double fl = ppm_face(a_2, a_1, a0, a1); /* value at i-1/2 */
        double fr = ppm_face(a_1, a0, a1, a2);  /* value at i+1/2 */
        double dp = fr - a0, dm = a0 - fl;
        if (dp * dm <= 0.0 || (a1 - a0) * (a0 - a_1) <= 0.0) {
            /* local extremum: extremum-preserving curvature limiter */
            double d2 = 6.0 * (fl - 2.0 * a0 + fr);
            double d2c = a_1 - 2.0 * a0 + a1;
            double d2l = a_2 - 2.0 * a_1 + a0;
            double d2r = a0 - 2.0 * a1 + a2;
            double lim = 0.0;
            if (d2 * d2c > 0.0 && d2 * d2l > 0.0 && d2 * d2r > 0.0) {
                double s = sgn_pos(d2);
                lim = s * dmin(dmin(PPM_C * fabs(d2l), PPM_C * fabs(d2r)),
                               dmin(PPM_C * fabs(d2c), fabs(d2)));
            }
            if (d2 != 0.0) {
                dp = dp * lim / d2;
                dm = dm * lim / d2;
            } else {
                dp = 0.0;
                dm = 0.0;
            }
        } else {
            /* monotone: remove overshoot of the parabola */
            if (fabs(dp) >= 2.0 * fabs(dm)) dp = 2.0 * dm;
            if (fabs(dm) >= 2.0 * fabs(dp)) dm = 2.0 * dp;
        }
        /* the limited interface values stay between the cell's and the
         * neighbour's characteristic values */
        double ar = dmax(dmin(a0, a1), dmin(a0 + dp, dmax(a0, a1)));
        double al = dmax(dmin(a0, a_1), dmin(a0 - dm, dmax(a0, a_1)));
        dplus[m] = ar - a0;
        dminus[m] = al - a0;
    }
    double wp[7], wm[7];
    matvec7(R, dplus, wp);
    matvec7(R, dminus, wm);
    const double *wl = w + 7, *wr = w + 21;
    for (int c = 0; c < 7; ++c) {
        double fp0 = w0[c] + wp[c];
        double fm0 = w0[c] + wm[c];
        /* bound the interface primitives between the neighbouring cell values */
        double fp = dmax(dmin(w0[c], wr[c]), dmin(fp0, dmax(w0[c], wr[c])));
        double fm = dmax(dmin(w0[c], wl[c]), dmin(fm0, dmax(w0[c], wl[c])));
        /* a bound that had to act (beyond rounding) marks a profile the
         * characteristic limiting did not keep monotone in this primitive:
         * its interface pair gets the Colella-Woodward monotonicity
         * constraints (flat at an extremum, otherwise the face beyond twice
         * the other's distance from the cell value is pulled back to it) */
        double tol = PPM_TIE * (fabs(w0[c]) + fabs(wl[c]) + fabs(wr[c]) + floor_c[c]);
        if (fabs(fp - fp0) > tol || fabs(fm - fm0) > tol) {
            double dpp = fp - w0[c], dmm = w0[c] - fm;
            if (dpp * dmm <= 0.0) {
                fp = w0[c];
                fm = w0[c];
            } else {
                if (fabs(dpp) >= 2.0 * fabs(dmm)) fp = w0[c] + 2.0 * dmm;
                if (fabs(dmm) >= 2.0 * fabs(dpp)) fm = w0[c] - 2.0 * dpp;
            }
        }
        face_plus[c] = fp;
        face_minus[c] = fm;
    }
}

/* ------------------------------------------------------------------------- */
/* Ghost-padded working grid and boundary mapping (Step 10: halo cells)       */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n[3];       /* interior cells */
    int p[3];       /* padded cells = n + 2*NG */
    int bc[3];
    double *u[5];   /* rho, mx, my, mz, E on padded cells */
    double *b[3];   /* face fields; axis d has p[d]+1 faces along d */
    double *w[8];   /* primitives rho, vx, vy, vz, P, Bcx, Bcy, Bcz */
} pgrid;

static int map_cell(int i, int n, int bc)
{
    if (bc == 0) return ((i % n) + n) % n;
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

static int map_face(int i, int n, int bc)
{
    if (bc == 0) return ((i % n) + n) % n;
    return i < 0 ? 0 : (i > n ? n : i);
}

/* padded cell index, i,j,k in [-NG, n+NG-1] */
static size_t pc(const pgrid *g, int i, int j, int k)
{
    return ((size_t)(k + NG) * g->p[1] + (size_t)(j + NG)) * g->p[0] + (size_t)(i + NG);
}

/* padded face index for axis d; the d-index runs over [-NG, n_d+NG] */
static size_t pf(const pgrid *g, int d, int i, int j, int k)
{
    int px = g->p[0] + (d == 0), py = g->p[1] + (d == 1);
    return ((size_t)(k + NG) * py + (size_t)(j + NG)) * px + (size_t)(i + NG);
}

static size_t ncell_padded(const pgrid *g) { return (size_t)g->p[0] * g->p[1] * g->p[2]; }
static size_t nface_padded(const pgrid *g, int d)
{
    return (size_t)(g->p[0] + (d == 0)) * (g->p[1] + (d == 1)) * (g->p[2] + (d == 2));
}

/* interior (unpadded) indices of the caller's arrays */
static size_t ic(const int n[3], int i, int j, int k)
{
    return ((size_t)k * n[1] + j) * n[0] + i;
}
static size_t ifc(const int n[3], int d, int i, int j, int k)
{
    int nx = n[0] + (d == 0), ny = n[1] + (d == 1);
    return ((size_t)k * ny + j) * nx + i;
}

static int pgrid_alloc(pgrid *g, const vref_grid *vg)
{
    memset(g, 0, sizeof(*g));
    g->n[0] = vg->nx; g->n[1] = vg->ny; g->n[2] = vg->nz;
    for (int d = 0; d < 3; ++d) {
        g->p[d] = g->n[d] + 2 * NG;
        g->bc[d] = vg->bc[d];
    }
    size_t nc = ncell_padded(g);
    for (int f = 0; f < 5; ++f) g->u[f] = (double *)malloc(nc * sizeof(double));
    for (int f = 0; f < 8; ++f) g->w[f] = (double *)malloc(nc * sizeof(double));
    for (int d = 0; d < 3; ++d) g->b[d] = (double *)malloc(nface_padded(g, d) * sizeof(double));
    for (int f = 0; f < 5; ++f) if (!g->u[f]) return 1;
    for (int f = 0; f < 8; ++f) if (!g->w[f]) return 1;
    for (int d = 0; d < 3; ++d) if (!g->b[d]) return 1;
    return 0;
}

static void pgrid_free(pgrid *g)
{
    for (int f = 0; f < 5; ++f) free(g->u[f]);
    for (int f = 0; f < 8; ++f) free(g->w[f]);
    for (int d = 0; d < 3; ++d) free(g->b[d]);
}

/* Fill the padded grid from a caller state by boundary index mapping. */
static void pgrid_fill(pgrid *g, const double *const st[8])
{
    const int *n = g->n;
    int k;
#pragma omp parallel for schedule(static)
    for (k = -NG; k < n[2] + NG; ++k)
        for (int j = -NG; j < n[1] + NG; ++j)
            for (int i = -NG; i < n[0] + NG; ++i) {
                size_t src = ic(n, map_cell(i, n[0], g->bc[0]), map_cell(j, n[1], g->bc[1]),
                                map_cell(k, n[2], g->bc[2]));
                size_t dst = pc(g, i, j, k);
                for (int f = 0; f < 5; ++f) g->u[f][dst] = st[f][src];
            }
    for (int d = 0; d < 3; ++d) {
        int lo[3] = {-NG, -NG, -NG};
        int hi[3] = {n[0] + NG - 1, n[1] + NG - 1, n[2] + NG - 1};
        hi[d] += 1;
#pragma omp parallel for schedule(static)
        for (k = lo[2]; k <= hi[2]; ++k)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    int idx[3] = {i, j, k}, m[3];
                    for (int e = 0; e < 3; ++e)
                        m[e] = (e == d) ? map_face(idx[e], n[e], g->bc[e])
                                        : map_cell(idx[e], n[e], g->bc[e]);
                    g->b[d][pf(g, d, i, j, k)] = st[5 + d][ifc(n, d, m[0], m[1], m[2])];
                }
    }
}

/* Primitive variables of every padded cell (Sec. 2.1; cell-centred B as the
 * average of the two face values, Sec. 2.2 Step 1). */
static uint32_t pgrid_prims(pgrid *g, double gamma)
{
    const int *n = g->n;
    uint32_t st = 0;
    int k;
#pragma omp parallel for schedule(static) reduction(| : st)
    for (k = -NG; k < n[2] + NG; ++k)
        for (int j = -NG; j < n[1] + NG; ++j)
            for (int i = -NG; i < n[0] + NG; ++i) {
                size_t c = pc(g, i, j, k);
                double bcx = 0.5 * (g->b[0][pf(g, 0, i, j, k)] + g->b[0][pf(g, 0, i + 1, j, k)]);
                double bcy = 0.5 * (g->b[1][pf(g, 1, i, j, k)] + g->b[1][pf(g, 1, i, j + 1, k)]);
                double bcz = 0.5 * (g->b[2][pf(g, 2, i, j, k)] + g->b[2][pf(g, 2, i, j, k + 1)]);
                double rho = g->u[0][c];
                if (!(rho >= FLOOR_RHO)) { rho = FLOOR_RHO; st |= VREF_STATUS_DENSITY_FLOOR; }
                double vx = g->u[1][c] / rho, vy = g->u[2][c] / rho, vz = g->u[3][c] / rho;
                double ke = 0.5 * rho * (vx * vx + vy * vy + vz * vz);
                double me = 0.5 * (bcx * bcx + bcy * bcy + bcz * bcz);
                double p = (gamma - 1.0) * (g->u[4][c] - ke - me);
                if (!(p >= FLOOR_P)) { p = FLOOR_P; st |= VREF_STATUS_PRESSURE_FLOOR; }
                g->w[0][c] = rho;
                g->w[1][c] = vx;
                g->w[2][c] = vy;
                g->w[3][c] = vz;
                g->w[4][c] = p;
                g->w[5][c] = bcx;
                g->w[6][c] = bcy;
                g->w[7][c] = bcz;
            }
    return st;
}

/* Sweep-frame 7-vector of a padded cell for direction d: (rho, v_n, v_t1,
 * v_t2, P, B_t1, B_t2) with (n, t1, t2) cyclic (Table emf note). */
static void frame_prim(const pgrid *g, size_t c, int d, double w[7])
{
    w[0] = g->w[0][c];
    w[1] = g->w[1 + d][c];
    w[2] = g->w[1 + (d + 1) % 3][c];
    w[3] = g->w[1 + (d + 2) % 3][c];
    w[4] = g->w[4][c];
    w[5] = g->w[5 + (d + 1) % 3][c];
    w[6] = g->w[5 + (d + 2) % 3][c];
}

static void step_cell(int d, int *i, int *j, int *k, int s)
{
    if (d == 0) *i += s; else if (d == 1) *j += s; else *k += s;
}

/* Face fluxes along axis d for every face whose reconstruction stencil lies
 * inside the padded grid.  F[c] is indexed like the padded face array of axis
 * d.  recon: 1 = PCM, 2 = PLMC, 3 = PPMC.  Returns floor status bits. */
static uint32_t stage_fluxes(const pgrid *g, int d, int recon, double gamma, double *F[8])
{
    const int *n = g->n;
    int r = recon == 1 ? 0 : ((recon == 2 || recon == 4) ? 1 : 2);
    size_t nc = ncell_padded(g);
    /* per-cell interface states: minus = low face, plus = high face */
    double *wm[7], *wp[7];
    for (int c = 0; c < 7; ++c) {
        wm[c] = (double *)malloc(nc * sizeof(double));
        wp[c] = (double *)malloc(nc * sizeof(double));
    }
    int lo[3] = {-NG, -NG, -NG}, hi[3] = {n[0] + NG - 1, n[1] + NG - 1, n[2] + NG - 1};
    lo[d] += r;
    hi[d] -= r;
    uint32_t st = 0;
    int k;
#pragma omp parallel for schedule(static) reduction(| : st)
    for (k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
            for (int i = lo[0]; i <= hi[0]; ++i) {
                size_t c0 = pc(g, i, j, k);
                double sten[35], fm[7], fp[7];
                for (int s = -r; s <= r; ++s) {
                    int ii = i, jj = j, kk = k;
                    step_cell(d, &ii, &jj, &kk, s);
                    frame_prim(g, pc(g, ii, jj, kk), d, sten + 7 * (s + r));
                }
                double bn_cc = g->w[5 + d][c0];
                if (r == 0) {
                    memcpy(fm, sten, sizeof(fm));
                    memcpy(fp, sten, sizeof(fp));
                } else if (recon == 2) {
                    vref_plmc(sten, bn_cc, gamma, fm, fp);
                } else if (recon == 4) {
                    vref_plmp(sten, fm, fp);
                } else if (recon == 3) {
                    vref_ppmc(sten, bn_cc, gamma, fm, fp);
                } else {
                    vref_ppmp(sten, bn_cc, gamma, fm, fp);
                }
                /* floors on reconstructed interface states */
                if (!(fm[0] >= FLOOR_RHO)) { fm[0] = FLOOR_RHO; st |= VREF_STATUS_DENSITY_FLOOR; }
                if (!(fp[0] >= FLOOR_RHO)) { fp[0] = FLOOR_RHO; st |= VREF_STATUS_DENSITY_FLOOR; }
                if (!(fm[4] >= FLOOR_P)) { fm[4] = FLOOR_P; st |= VREF_STATUS_PRESSURE_FLOOR; }
                if (!(fp[4] >= FLOOR_P)) { fp[4] = FLOOR_P; st |= VREF_STATUS_PRESSURE_FLOOR; }
                for (int c = 0; c < 7; ++c) {
                    wm[c][c0] = fm[c];
                    wp[c][c0] = fp[c];
                }
            }
    /* faces: face f on axis d lies between cells f-1 and f */
    int flo[3] = {-NG, -NG, -NG}, fhi[3] = {n[0] + NG - 1, n[1] + NG - 1, n[2] + NG - 1};
    flo[d] = -NG + r + 1;
    fhi[d] = n[d] + NG - 1 - r;
#pragma omp parallel for schedule(static)
    for (k = flo[2]; k <= fhi[2]; ++k)
        for (int j = flo[1]; j <= fhi[1]; ++j)
            for (int i = flo[0]; i <= fhi[0]; ++i) {
                int il = i, jl = j, kl = k;
                step_cell(d, &il, &jl, &kl, -1);
                size_t cl = pc(g, il, jl, kl), cr = pc(g, i, j, k);
                double wl[7], wr[7], f[8];
                for (int c = 0; c < 7; ++c) {
                    wl[c] = wp[c][cl];
                    wr[c] = wm[c][cr];
                }
                double bn = g->b[d][pf(g, d, i, j, k)];
                vref_hlld(wl, wr, bn, gamma, f);
                size_t fi = pf(g, d, i, j, k);
                for (int c = 0; c < 8; ++c) F[c][fi] = f[c];
            }
    for (int c = 0; c < 7; ++c) {
        free(wm[c]);
        free(wp[c]);
    }
    return st;
}

/* ------------------------------------------------------------------------- */
/* Constrained transport (Sec. 2.2 Step 4, Table emf, Eqs. emf-edge,          */
/* emf-upwind-slope, emf-slope and the reference field E_ref = -v x B)        */
/* ------------------------------------------------------------------------- */

/* Face EMF component `comp` (0 = x, 1 = y, 2 = z) carried by the flux of a
 * face normal to axis d (Table emf): E_{t2} = -F[B_t1], E_{t1} = +F[B_t2]. */
static double face_emf(double *const F[3][8], int d, int comp, size_t fi)
{
    int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    if (comp == t2) return -F[d][5][fi];
    if (comp == t1) return F[d][6][fi];
    return 0.0;
}

/* Cell reference EMF component `comp`: E_ref = -(v x B_cc). */
static double ref_emf(const pgrid *g, size_t c, int comp)
{
    double vx = g->w[1][c], vy = g->w[2][c], vz = g->w[3][c];
    double bx = g->w[5][c], by = g->w[6][c], bz = g->w[7][c];
    if (comp == 0) return -(vy * bz - vz * by);
    if (comp == 1) return -(vz * bx - vx * bz);
    return -(vx * by - vy * bx);
}

static double upwind(double s, double lo, double hi)
{
    if (s > 0.0) return lo;
    if (s < 0.0) return hi;
    return 0.5 * (lo + hi);
}

/* Edge EMF along axis a at the edge whose two transverse coordinates (axes
 * b = a+1, c = a+2) are at the low faces of cell (i,j,k); e.g. a = z gives
 * E_z(i-1/2, j-1/2, k). */
static double edge_emf(const pgrid *g, double *const F[3][8], int a, int i, int j, int k)
{
    int b = (a + 1) % 3, c = (a + 2) % 3;
    int x0[3] = {i, j, k};
    /* cells around the edge: (b-1|b, c-1|c) */
    int cb[3], cc_[3], cbc[3];
    memcpy(cb, x0, sizeof(cb));
    cb[b] -= 1;                 /* (b-1, c)   */
    memcpy(cc_, x0, sizeof(cc_));
    cc_[c] -= 1;                /* (b, c-1)   */
    memcpy(cbc, x0, sizeof(cbc));
    cbc[b] -= 1;
    cbc[c] -= 1;                /* (b-1, c-1) */
    size_t c00 = pc(g, x0[0], x0[1], x0[2]);     /* (b, c)     */
    size_t c10 = pc(g, cb[0], cb[1], cb[2]);     /* (b-1, c)   */
    size_t c01 = pc(g, cc_[0], cc_[1], cc_[2]);  /* (b, c-1)   */
    size_t c11 = pc(g, cbc[0], cbc[1], cbc[2]);  /* (b-1, c-1) */
    /* b-faces at (b-1/2, c) and (b-1/2, c-1): face index = cell (b, .) */
    size_t fb_c = pf(g, b, x0[0], x0[1], x0[2]);
    size_t fb_cm = pf(g, b, cc_[0], cc_[1], cc_[2]);
    /* c-faces at (b, c-1/2) and (b-1, c-1/2) */
    size_t fc_b = pf(g, c, x0[0], x0[1], x0[2]);
    size_t fc_bm = pf(g, c, cb[0], cb[1], cb[2]);

    double eb_c = face_emf(F, b, a, fb_c), eb_cm = face_emf(F, b, a, fb_cm);
    double ec_b = face_emf(F, c, a, fc_b), ec_bm = face_emf(F, c, a, fc_bm);
    double r00 = ref_emf(g, c00, a), r10 = ref_emf(g, c10, a);
    double r01 = ref_emf(g, c01, a), r11 = ref_emf(g, c11, a);
    double sb_c = F[b][7][fb_c], sb_cm = F[b][7][fb_cm];  /* upwind indicators */
    double sc_b = F[c][7][fc_b], sc_bm = F[c][7][fc_bm];

    double avg = 0.25 * (eb_c + eb_cm + ec_b + ec_bm);
    /* slopes towards the edge along c, taken from the c-faces, upwinded along b */
    double t1 = upwind(sb_c, ec_bm - r10, ec_b - r00);
    double t2 = upwind(sb_cm, ec_bm - r11, ec_b - r01);
    /* slopes towards the edge along b, taken from the b-faces, upwinded along c */
    double t3 = upwind(sc_b, eb_cm - r01, eb_c - r00);
    double t4 = upwind(sc_bm, eb_cm - r11, eb_c - r10);
    return avg + 0.25 * (t1 + t2 + t3 + t4);
}

/* Edge arrays (interior + boundary edges):
 *  ex (nz+1)*(ny+1)*nx, ey (nz+1)*ny*(nx+1), ez nz*(ny+1)*(nx+1). */
static size_t edge_index(const int n[3], int a, int i, int j, int k)
{
    int ex[3] = {n[0] + (a != 0), n[1] + (a != 1), n[2] + (a != 2)};
    return ((size_t)k * ex[1] + j) * ex[0] + i;
}

static size_t edge_count(const int n[3], int a)
{
    return (size_t)(n[0] + (a != 0)) * (n[1] + (a != 1)) * (n[2] + (a != 2));
}

static void stage_edges(const pgrid *g, double *const F[3][8], double *E[3])
{
    const int *n = g->n;
    for (int a = 0; a < 3; ++a) {
        int hi[3] = {n[0] - 1 + (a != 0), n[1] - 1 + (a != 1), n[2] - 1 + (a != 2)};
        int k;
#pragma omp parallel for schedule(static)
        for (k = 0; k <= hi[2]; ++k)
            for (int j = 0; j <= hi[1]; ++j)
                for (int i = 0; i <= hi[0]; ++i)
                    E[a][edge_index(n, a, i, j, k)] = edge_emf(g, F, a, i, j, k);
    }
}

/* Conservative update of the cell variables (Sec. 2.2 Steps 5/9):
 * out = base - dt/dx (F_x(i+1/2)-F_x(i-1/2)) - dt/dy (...) - dt/dz (...). */
static void stage_update_cells(const pgrid *g, double *const F[3][8], const double *const base[8],
                               double *const out[8], double dt, const double dl[3])
{
    const int *n = g->n;
    double c[3] = {dt / dl[0], dt / dl[1], dt / dl[2]};
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                size_t id = ic(n, i, j, k);
                double acc[5];
                for (int f = 0; f < 5; ++f) acc[f] = base[f][id];
                for (int d = 0; d < 3; ++d) {
                    int ip = i, jp = j, kp = k;
                    step_cell(d, &ip, &jp, &kp, 1);
                    size_t flo = pf(g, d, i, j, k), fhi = pf(g, d, ip, jp, kp);
                    /* sweep-frame momentum components back to x, y, z */
                    int mcomp[3] = {1 + d, 1 + (d + 1) % 3, 1 + (d + 2) % 3};
                    double dF[5];
                    dF[0] = F[d][0][fhi] - F[d][0][flo];
                    dF[4] = F[d][4][fhi] - F[d][4][flo];
                    for (int m = 0; m < 3; ++m)
                        dF[mcomp[m]] = F[d][1 + m][fhi] - F[d][1 + m][flo];
                    for (int f = 0; f < 5; ++f) acc[f] = acc[f] - c[d] * dF[f];
                }
                for (int f = 0; f < 5; ++f) out[f][id] = acc[f];
            }
}

/* Face update B = B0 - dt curl(E) (Sec. 2.2 Steps 5/9).  On periodic axes the
 * duplicated last face is a copy of face 0. */
static void ct_update_faces(const int n[3], const int bc[3], const double *const b0[3],
                            double *const bout[3], const double *const E[3], double dt,
                            const double dl[3])
{
    for (int d = 0; d < 3; ++d) {
        int e1 = (d + 1) % 3, e2 = (d + 2) % 3;  /* curl_d = dE_e2/de1 - dE_e1/de2 */
        int hi[3] = {n[0] - 1, n[1] - 1, n[2] - 1};
        hi[d] = bc[d] == 0 ? n[d] - 1 : n[d];
        double c1 = dt / dl[e1], c2 = dt / dl[e2];
        int k;
#pragma omp parallel for schedule(static)
        for (k = 0; k <= hi[2]; ++k)
            for (int j = 0; j <= hi[1]; ++j)
                for (int i = 0; i <= hi[0]; ++i) {
                    int x[3] = {i, j, k};
                    int xp1[3] = {i, j, k}, xp2[3] = {i, j, k};
                    xp1[e1] += 1;
                    xp2[e2] += 1;
                    /* E_e2 on the edges at e1 -/+ 1/2, E_e1 on the edges at e2 -/+ 1/2 */
                    double de2 = E[e2][edge_index(n, e2, xp1[0], xp1[1], xp1[2])]
                                 - E[e2][edge_index(n, e2, x[0], x[1], x[2])];
                    double de1 = E[e1][edge_index(n, e1, xp2[0], xp2[1], xp2[2])]
                                 - E[e1][edge_index(n, e1, x[0], x[1], x[2])];
                    size_t fi = ifc(n, d, i, j, k);
                    bout[d][fi] = b0[d][fi] - c1 * de2 + c2 * de1;
                }
        if (bc[d] == 0) {
            /* duplicate plane n_d = plane 0 */
            int lo2[3] = {0, 0, 0}, hi2[3] = {n[0] - 1, n[1] - 1, n[2] - 1};
            lo2[d] = hi2[d] = 0;
            for (int k2 = lo2[2]; k2 <= hi2[2]; ++k2)
                for (int j2 = lo2[1]; j2 <= hi2[1]; ++j2)
                    for (int i2 = lo2[0]; i2 <= hi2[0]; ++i2) {
                        int xs[3] = {i2, j2, k2};
                        int xd[3] = {i2, j2, k2};
                        xd[d] = n[d];
                        bout[d][ifc(n, d, xd[0], xd[1], xd[2])] =
                            bout[d][ifc(n, d, xs[0], xs[1], xs[2])];
                    }
        }
    }
}

void vref_ct_update(const vref_grid *vg, const double *const b_in[3], double *const b_out[3],
                    const double *ex, const double *ey, const double *ez, double dt)
{
    int n[3] = {vg->nx, vg->ny, vg->nz};
    double dl[3] = {vg->dx, vg->dy, vg->dz};
    const double *E[3] = {ex, ey, ez};
    ct_update_faces(n, vg->bc, b_in, b_out, E, dt, dl);
}

/* ------------------------------------------------------------------------- */
/* Stage driver                                                               */
/* ------------------------------------------------------------------------- */

typedef struct {
    double *F[3][8];   /* 7 flux components + upwind indicator per face */
    double *E[3];
} stage_buf;

static int stage_alloc(stage_buf *s, const pgrid *g)
{
    memset(s, 0, sizeof(*s));
    for (int d = 0; d < 3; ++d) {
        size_t nf = nface_padded(g, d);
        for (int c = 0; c < 8; ++c) {
            s->F[d][c] = (double *)calloc(nf, sizeof(double));
            if (!s->F[d][c]) return 1;
        }
        s->E[d] = (double *)calloc(edge_count(g->n, d), sizeof(double));
        if (!s->E[d]) return 1;
    }
    return 0;
}

static void stage_free(stage_buf *s)
{
    for (int d = 0; d < 3; ++d) {
        for (int c = 0; c < 8; ++c) free(s->F[d][c]);
        free(s->E[d]);
    }
}

/* Fluxes + edge EMFs of a stage state `st`. */
static uint32_t stage_compute(pgrid *g, stage_buf *s, const double *const st[8], int recon,
                              double gamma)
{
    pgrid_fill(g, st);
    uint32_t status = pgrid_prims(g, gamma);
    for (int d = 0; d < 3; ++d) status |= stage_fluxes(g, d, recon, gamma, s->F[d]);
    stage_edges(g, s->F, s->E);
    return status;
}

static int grid_ok(const vref_grid *g)
{
    if (!g) return 0;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return 0;
    if (!(g->dx > 0.0) || !(g->dy > 0.0) || !(g->dz > 0.0)) return 0;
    if (!(g->gamma > 1.0)) return 0;
    if (!(g->cfl > 0.0 && g->cfl <= 0.5)) return 0;
    if (g->recon < 1 || g->recon > 5) return 0;
    for (int d = 0; d < 3; ++d)
        if (g->bc[d] != 0 && g->bc[d] != 1) return 0;
    return 1;
}

static size_t field_len(const vref_grid *g, int f)
{
    size_t nx = g->nx, ny = g->ny, nz = g->nz;
    if (f < 5) return nx * ny * nz;
    if (f == 5) return (nx + 1) * ny * nz;
    if (f == 6) return nx * (ny + 1) * nz;
    return nx * ny * (nz + 1);
}

/* CFL step of a state (Sec. 2.2 Step 1, Eq. dt): dt = C / max over cells and
 * directions of (|v_l| + c_f,l) / d_l, c_f,l from cell-centred values with
 * B_l as the longitudinal field. */
static double cfl_from_state(const vref_grid *vg, const double *const st[8], uint32_t *status)
{
    int n[3] = {vg->nx, vg->ny, vg->nz};
    double dl[3] = {vg->dx, vg->dy, vg->dz};
    double gmax = 0.0;
    uint32_t stb = 0;
    int k;
#pragma omp parallel for schedule(static) reduction(max : gmax) reduction(| : stb)
    for (k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                size_t c = ic(n, i, j, k);
                /* the high faces go through the face map: on a periodic axis the
                 * stored duplicate of face 0 is not read */
                int ip = map_face(i + 1, n[0], vg->bc[0]);
                int jp = map_face(j + 1, n[1], vg->bc[1]);
                int kp = map_face(k + 1, n[2], vg->bc[2]);
                double bc[3];
                bc[0] = 0.5 * (st[5][ifc(n, 0, i, j, k)] + st[5][ifc(n, 0, ip, j, k)]);
                bc[1] = 0.5 * (st[6][ifc(n, 1, i, j, k)] + st[6][ifc(n, 1, i, jp, k)]);
                bc[2] = 0.5 * (st[7][ifc(n, 2, i, j, k)] + st[7][ifc(n, 2, i, j, kp)]);
                double rho = st[0][c];
                if (!(rho >= FLOOR_RHO)) { rho = FLOOR_RHO; stb |= VREF_STATUS_DENSITY_FLOOR; }
                double v[3] = {st[1][c] / rho, st[2][c] / rho, st[3][c] / rho};
                double ke = 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                double me = 0.5 * (bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
                double p = (vg->gamma - 1.0) * (st[4][c] - ke - me);
                if (!(p >= FLOOR_P)) { p = FLOOR_P; stb |= VREF_STATUS_PRESSURE_FLOOR; }
                for (int d = 0; d < 3; ++d) {
                    double cf = fast_speed(rho, p, bc[d], bc[(d + 1) % 3], bc[(d + 2) % 3],
                                           vg->gamma);
                    double r = (fabs(v[d]) + cf) / dl[d];
                    if (r > gmax) gmax = r;
                }
            }
    if (status) *status |= stb;
    return vg->cfl / gmax;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int vref_cfl_dt(const vref_grid *g, const double *const st[8], double *dt, int nthreads)
{
    if (!grid_ok(g) || !st || !dt) return VREF_EINVAL;
    set_threads(nthreads);
    *dt = cfl_from_state(g, st, NULL);
    return VREF_OK;
}

/* One VL+CT step (Sec. 2.2 Steps 2-9; Step 1's dt is an input and the next
 * step's dt is computed from the result). */
int vref_step(const vref_grid *vg, const double *const in[8], double *const out[8],
              double dt, double *next_dt, uint32_t *status, int nthreads)
{
    if (!grid_ok(vg) || !in || !out || !(dt > 0.0) || !isfinite(dt)) return VREF_EINVAL;
    for (int f = 0; f < 8; ++f)
        if (!in[f] || !out[f]) return VREF_EINVAL;
    set_threads(nthreads);
    int n[3] = {vg->nx, vg->ny, vg->nz};
    double dl[3] = {vg->dx, vg->dy, vg->dz};

    pgrid g;
    stage_buf s;
    double *half[8], *base[8];
    int err = pgrid_alloc(&g, vg);
    err |= stage_alloc(&s, &g);
    for (int f = 0; f < 8; ++f) {
        half[f] = (double *)malloc(field_len(vg, f) * sizeof(double));
        base[f] = (double *)malloc(field_len(vg, f) * sizeof(double));
        if (!half[f] || !base[f]) err = 1;
    }
    uint32_t st = 0;
    if (!err) {
        /* keep U^n: out may alias in */
        for (int f = 0; f < 8; ++f) memcpy(base[f], in[f], field_len(vg, f) * sizeof(double));
        const double *const *b0 = (const double *const *)base;

        /* predictor: PCM + HLLD (Steps 2-3), CT EMFs (Step 4), half update (Step 5) */
        st |= stage_compute(&g, &s, b0, 1, vg->gamma);
        stage_update_cells(&g, s.F, b0, half, 0.5 * dt, dl);
        ct_update_faces(n, vg->bc, b0 + 5, half + 5, (const double *const *)s.E, 0.5 * dt, dl);

        /* corrector: reconstruction + HLLD (Steps 6-7), CT EMFs of the half
         * state (Step 8), full update from U^n (Step 9) */
        st |= stage_compute(&g, &s, (const double *const *)half, vg->recon, vg->gamma);
        stage_update_cells(&g, s.F, b0, out, dt, dl);
        ct_update_faces(n, vg->bc, b0 + 5, out + 5, (const double *const *)s.E, dt, dl);

        for (int f = 0; f < 8; ++f) {
            size_t len = field_len(vg, f);
            for (size_t q = 0; q < len; ++q)
                if (!isfinite(out[f][q])) { st |= VREF_STATUS_NONFINITE; break; }
        }
        if (next_dt) *next_dt = cfl_from_state(vg, (const double *const *)out, &st);
    }
    for (int f = 0; f < 8; ++f) {
        free(half[f]);
        free(base[f]);
    }
    stage_free(&s);
    pgrid_free(&g);
    if (status) *status |= st;
    return err ? VREF_EINVAL : VREF_OK;
}

int vref_edge_emfs(const vref_grid *vg, const double *const st[8], int recon, double *ex,
                   double *ey, double *ez, int nthreads)
{
    if (!grid_ok(vg) || !st || recon < 1 || recon > 5) return VREF_EINVAL;
    set_threads(nthreads);
    pgrid g;
    stage_buf s;
    int err = pgrid_alloc(&g, vg);
    err |= stage_alloc(&s, &g);
    if (!err) {
        stage_compute(&g, &s, st, recon, vg->gamma);
        memcpy(ex, s.E[0], edge_count(g.n, 0) * sizeof(double));
        memcpy(ey, s.E[1], edge_count(g.n, 1) * sizeof(double));
        memcpy(ez, s.E[2], edge_count(g.n, 2) * sizeof(double));
    }
    stage_free(&s);
    pgrid_free(&g);
    return err ? VREF_EINVAL : VREF_OK;
}

double vref_divb_norm(const vref_grid *vg, const double *const st[8])
{
    int n[3] = {vg->nx, vg->ny, vg->nz};
    double dl[3] = {vg->dx, vg->dy, vg->dz};
    double dmaxv = 0.0, bmax = 0.0;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                double d = (st[5][ifc(n, 0, i + 1, j, k)] - st[5][ifc(n, 0, i, j, k)]) / dl[0]
                           + (st[6][ifc(n, 1, i, j + 1, k)] - st[6][ifc(n, 1, i, j, k)]) / dl[1]
                           + (st[7][ifc(n, 2, i, j, k + 1)] - st[7][ifc(n, 2, i, j, k)]) / dl[2];
                if (fabs(d) > dmaxv) dmaxv = fabs(d);
                double bx = 0.5 * (st[5][ifc(n, 0, i + 1, j, k)] + st[5][ifc(n, 0, i, j, k)]);
                double by = 0.5 * (st[6][ifc(n, 1, i, j + 1, k)] + st[6][ifc(n, 1, i, j, k)]);
                double bz = 0.5 * (st[7][ifc(n, 2, i, j, k + 1)] + st[7][ifc(n, 2, i, j, k)]);
                double b = sqrt(bx * bx + by * by + bz * bz);
                if (b > bmax) bmax = b;
            }
    if (bmax == 0.0) return dmaxv == 0.0 ? 0.0 : INFINITY;
    return dmaxv * dl[0] / bmax;
}

/* Predictor only (Sec. 2.2 Steps 2-5): the half-step state U^{n+1/2} of a
 * step of size dt (diagnostics and stage-level pins). */
int vref_half_step(const vref_grid *vg, const double *const in[8], double *const out[8],
                   double dt, int nthreads)
{
    if (!grid_ok(vg) || !in || !out || !(dt > 0.0)) return VREF_EINVAL;
    set_threads(nthreads);
    int n[3] = {vg->nx, vg->ny, vg->nz};
    double dl[3] = {vg->dx, vg->dy, vg->dz};
    pgrid g;
    stage_buf s;
    int err = pgrid_alloc(&g, vg);
    err |= stage_alloc(&s, &g);
    if (!err) {
        stage_compute(&g, &s, in, 1, vg->gamma);
        stage_update_cells(&g, s.F, in, out, 0.5 * dt, dl);
        ct_update_faces(n, vg->bc, in + 5, out + 5, (const double *const *)s.E, 0.5 * dt, dl);
    }
    stage_free(&s);
    pgrid_free(&g);
    return err ? VREF_EINVAL : VREF_OK;
}

/* Face fluxes of one stage (diagnostics): for a state `st` and reconstruction
 * `recon`, writes the 7 sweep-frame flux components and the upwind indicator
 * of every face of axis d into F[d] (8 arrays, face layout of the state's
 * normal field on axis d). */
int vref_stage_fluxes(const vref_grid *vg, const double *const st[8], int recon,
                      double *const Fx[8], double *const Fy[8], double *const Fz[8], int nthreads)
{
    if (!grid_ok(vg) || !st || recon < 1 || recon > 5) return VREF_EINVAL;
    set_threads(nthreads);
    pgrid g;
    stage_buf s;
    int err = pgrid_alloc(&g, vg);
    err |= stage_alloc(&s, &g);
    double *const *F[3] = {Fx, Fy, Fz};
    if (!err) {
        stage_compute(&g, &s, st, recon, vg->gamma);
        for (int d = 0; d < 3; ++d) {
            int hi[3] = {g.n[0] - 1, g.n[1] - 1, g.n[2] - 1};
            hi[d] = g.n[d];
            for (int k = 0; k <= hi[2]; ++k)
                for (int j = 0; j <= hi[1]; ++j)
                    for (int i = 0; i <= hi[0]; ++i)
                        for (int c = 0; c < 8; ++c)
                            F[d][c][ifc(g.n, d, i, j, k)] = s.F[d][c][pf(&g, d, i, j, k)];
        }
    }
    stage_free(&s);
    pgrid_free(&g);
    return err ? VREF_EINVAL : VREF_OK;
}
