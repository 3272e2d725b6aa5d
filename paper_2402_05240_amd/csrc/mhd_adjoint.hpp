// mhd_adjoint.hpp -- reverse derivatives of the per-state physics of
// mhd_physics.hpp (Caddy & Schneider, "Cholla-MHD", Sec. 2.2 Steps 3 and 6):
// HLLD, the characteristic eigen-system with its projections, and the PLMC /
// PLMP reconstructions.  Each function re-evaluates its forward formulas in
// FP64 (same operations, so the same branches), then applies the chain rule in
// reverse order.  Every branch of the forward evaluation (wave-speed min/max,
// HLLD fan region and degeneracy fallback, noise snapping, limiter choice,
// clamps) is held fixed: the result is the derivative of the branch taken.
// Naming: a_x is the cotangent (adjoint) of the forward quantity x.
#pragma once
#include "mhd_physics.hpp"

namespace vlct {

// forward choice of fmin / fmax: true when the second argument is returned
VLCT_DEV bool takes_second_min(double a, double b) { return b < a; }
VLCT_DEV bool takes_second_max(double a, double b) { return b > a; }
// derivative of |x| on the branch taken (+1 at x = 0)
VLCT_DEV double abs_slope(double x) { return x < 0.0 ? -1.0 : 1.0; }
VLCT_DEV double sqrt_slope(double r) { return r > 0.0 ? 0.5 / r : 0.0; }  // d sqrt(q) / dq at r = sqrt(q)

// ---------------------------------------------------------------------------
// fast speed: cf2 = (gP + B^2 + disc) / (2 rho), disc = sqrt((gP - B^2)^2 + 4 gP B_perp^2)
// ---------------------------------------------------------------------------
struct FastSq {
    double gp, bp2, b2, t, disc, cf2;
};

// the terms of cf2 up to the numerator gP + B^2 + disc
VLCT_DEV FastSq fast_sq_terms(double p, double bn2, double bt1, double bt2, double gam)
{
    FastSq q;
    q.gp = gam * p;
    q.bp2 = bt1 * bt1 + bt2 * bt2;
    q.b2 = bn2 + q.bp2;
    q.t = q.gp - q.b2;
    q.disc = msqrt(q.t * q.t + 4.0 * q.gp * q.bp2);
    q.cf2 = 0.0;
    return q;
}

// adds the cotangents of (d, p, bn, bt1, bt2) given those of cf2 and disc;
// i2d = 1 / (2 rho), idc = 1 / disc (read only where disc > 0)
VLCT_DEV void fast_sq_rev(const FastSq &q, double i2d, double idc, double bn, double bt1,
                          double bt2, double gam, double a_cf2, double a_disc, double &a_d,
                          double &a_p, double &a_bn, double &a_bt1, double &a_bt2)
{
    double a_gp = a_cf2 * i2d;
    double a_b2 = a_cf2 * i2d;
    a_disc = a_disc + a_cf2 * i2d;
    a_d = a_d - a_cf2 * q.cf2 * (2.0 * i2d);  // d cf2 / d rho = -cf2 / rho
    double a_bp2 = 0.0;
    if (q.disc > 0.0) {
        const double a_t = a_disc * q.t * idc;
        a_gp = a_gp + a_disc * 2.0 * q.bp2 * idc + a_t;
        a_bp2 = a_disc * 2.0 * q.gp * idc;
        a_b2 = a_b2 - a_t;
    }
    a_bn = a_bn + 2.0 * bn * a_b2;
    a_bp2 = a_bp2 + a_b2;
    a_bt1 = a_bt1 + 2.0 * bt1 * a_bp2;
    a_bt2 = a_bt2 + 2.0 * bt2 * a_bp2;
    a_p = a_p + gam * a_gp;
}

// ---------------------------------------------------------------------------
// HLLD reverse: (a_L, a_R, a_bn) += J^T a_f, J = d f / d(L, R, bn) of hlld()
// ---------------------------------------------------------------------------
VLCT_DEV void hlld_rev(const W7 &L, const W7 &R, double bn, double gam, double gm1i,
                       const double a_f[7], W7 &aL, W7 &aR, double &a_bn_out)
{
    // ---- forward (the formulas of hlld(), intermediates kept)
    const double bn2 = bn * bn;
    const double pbL = 0.5 * (bn2 + L.by * L.by + L.bz * L.bz);
    const double pbR = 0.5 * (bn2 + R.by * R.by + R.bz * R.bz);
    const double ptL = L.p + pbL;
    const double ptR = R.p + pbR;
    const double u2L = L.u * L.u + L.v * L.v + L.w * L.w;
    const double u2R = R.u * R.u + R.v * R.v + R.w * R.w;
    const double eL = L.p * gm1i + 0.5 * L.d * u2L + pbL;
    const double eR = R.p * gm1i + 0.5 * R.d * u2R + pbR;
    // c_f = num rq, rq = 1 / sqrt(2 rho num), num = gP + B^2 + disc; then
    // 1 / c_f = 2 rho rq and 1 / (2 rho) = num rq^2
    auto fast_fwd = [&](const W7 &X, FastSq &q, double &rq) {
        q = fast_sq_terms(X.p, bn2, X.by, X.bz, gam);
        const double num = q.gp + q.b2 + q.disc;
        rq = mrsqrt(2.0 * X.d * num);
        q.cf2 = num * (num * rq * rq);
        return num * rq;
    };
    double cfL, cfR;
    {
        FastSq q;
        double rq;
        cfL = fast_fwd(L, q, rq);
        cfR = fast_fwd(R, q, rq);
    }
    const bool cmaxR = takes_second_max(cfL, cfR);
    const double cmax = cmaxR ? cfR : cfL;
    const bool uminR = takes_second_min(L.u, R.u);
    const bool umaxR = takes_second_max(L.u, R.u);
    const double sL = (uminR ? R.u : L.u) - cmax;
    const double sR = (umaxR ? R.u : L.u) + cmax;
    const double qL = (sL - L.u) * L.d;
    const double qR = (sR - R.u) * R.d;
    const double iq = 1.0 / (qR - qL);
    const double num_m = qR * R.u - qL * L.u - ptR + ptL;
    const double sM = num_m * iq;
    const double num_p = qR * ptL - qL * ptR + qL * qR * (R.u - L.u);
    const double pts = num_p * iq;

    double su[2], ssm[2], issm[2], ds[2], den[2], iden[2], t1[2], t2[2];
    double vs[2], ws[2], bys[2], bzs[2], vbs[2], vb[2], num_e[2], es[2];
    bool degen[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const W7 &X = a == 0 ? L : R;
        const double S = a == 0 ? sL : sR;
        const double pt = a == 0 ? ptL : ptR;
        const double e = a == 0 ? eL : eR;
        su[a] = S - X.u;
        ssm[a] = S - sM;
        issm[a] = 1.0 / ssm[a];
        ds[a] = X.d * su[a] * issm[a];
        den[a] = X.d * su[a] * ssm[a] - bn2;
        degen[a] = fabs(den[a]) < kHlldDegen * pts;
        iden[a] = 1.0 / den[a];
        t1[a] = degen[a] ? 0.0 : bn * (sM - X.u) * iden[a];
        t2[a] = degen[a] ? 1.0 : (X.d * su[a] * su[a] - bn2) * iden[a];
        vs[a] = X.v - X.by * t1[a];
        ws[a] = X.w - X.bz * t1[a];
        bys[a] = X.by * t2[a];
        bzs[a] = X.bz * t2[a];
        vbs[a] = sM * bn + vs[a] * bys[a] + ws[a] * bzs[a];
        vb[a] = X.u * bn + X.v * X.by + X.w * X.bz;
        num_e[a] = su[a] * e - pt * X.u + pts * sM + bn * (vb[a] - vbs[a]);
        es[a] = num_e[a] * issm[a];
    }
    const double sg = bn >= 0.0 ? 1.0 : -1.0;
    const double irL = mrsqrt(ds[0]), irR = mrsqrt(ds[1]);
    const double rL = ds[0] * irL, rR = ds[1] * irR;
    const double isum = 1.0 / (rL + rR);
    const double nv = rL * vs[0] + rR * vs[1] + sg * (bys[1] - bys[0]);
    const double nw = rL * ws[0] + rR * ws[1] + sg * (bzs[1] - bzs[0]);
    const double nby = rL * bys[1] + rR * bys[0] + sg * rL * rR * (vs[1] - vs[0]);
    const double nbz = rL * bzs[1] + rR * bzs[0] + sg * rL * rR * (ws[1] - ws[0]);
    const double vss = nv * isum, wss = nw * isum, byss = nby * isum, bzss = nbz * isum;
    const double vbss = sM * bn + vss * byss + wss * bzss;

    const bool left = sM >= 0.0;
    const W7 &X = left ? L : R;
    const double S = left ? sL : sR;
    const double pt = left ? ptL : ptR;
    const double e = left ? eL : eR;
    const double r = left ? rL : rR;
    const double car = fabs(bn) * (left ? irL : irR);
    const double ss = left ? sM - car : sM + car;
    const bool star_only = left ? (ss >= 0.0) : (ss <= 0.0);
    const double vbs_a = left ? vbs[0] : vbs[1];
    const double ess = left ? es[0] - r * sg * (vbs[0] - vbss) : es[1] + r * sg * (vbs[1] - vbss);
    const bool outer = left ? (sL > 0.0) : (sR < 0.0);
    const double cS = outer ? 0.0 : S;
    const double cSS = (outer || star_only) ? 0.0 : ss;
    const double vbX = left ? vb[0] : vb[1];
    const double mu = X.d * X.u;
    const double dsa = left ? ds[0] : ds[1];
    const double vsa = left ? vs[0] : vs[1], wsa = left ? ws[0] : ws[1];
    const double bysa = left ? bys[0] : bys[1], bzsa = left ? bzs[0] : bzs[1];
    const double esa = left ? es[0] : es[1];
    const double dU[7] = {dsa - X.d, dsa * sM - mu, dsa * vsa - X.d * X.v, dsa * wsa - X.d * X.w,
                          esa - e, bysa - X.by, bzsa - X.bz};
    const double dV[7] = {0.0, 0.0, dsa * (vss - vsa), dsa * (wss - wsa), ess - esa, byss - bysa,
                          bzss - bzsa};

    // ---- reverse
    // cotangents of the chosen side's state X and of shared quantities
    double aXd = 0.0, aXu = 0.0, aXv = 0.0, aXw = 0.0, aXby = 0.0, aXbz = 0.0;
    double a_bn = 0.0, a_bn2 = 0.0, a_sM = 0.0, a_pts = 0.0;
    double a_ptX = 0.0, a_eX = 0.0, a_S = 0.0;
    double a_ds[2] = {0.0, 0.0}, a_vs[2] = {0.0, 0.0}, a_ws[2] = {0.0, 0.0};
    double a_bys[2] = {0.0, 0.0}, a_bzs[2] = {0.0, 0.0}, a_es[2] = {0.0, 0.0};
    double a_vbs[2] = {0.0, 0.0};
    double a_vss = 0.0, a_wss = 0.0, a_byss = 0.0, a_bzss = 0.0, a_ess = 0.0, a_ss = 0.0;
    double a_rL = 0.0, a_rR = 0.0;

    double a_cS = 0.0, a_cSS = 0.0;
#pragma unroll
    for (int k = 0; k < 7; ++k) a_cS = a_cS + a_f[k] * dU[k];
#pragma unroll
    for (int k = 2; k < 7; ++k) a_cSS = a_cSS + a_f[k] * dV[k];
    if (!outer) a_S = a_S + a_cS;
    if (!(outer || star_only)) a_ss = a_ss + a_cSS;
    double a_dU[7], a_dV[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        a_dU[k] = cS * a_f[k];
        a_dV[k] = cSS * a_f[k];
    }
    double a_dsa = 0.0, a_vsa = 0.0, a_wsa = 0.0, a_esa = 0.0, a_bysa = 0.0, a_bzsa = 0.0;
    double a_mu = 0.0;
    // dV
    a_dsa = a_dsa + a_dV[2] * (vss - vsa) + a_dV[3] * (wss - wsa);
    a_vss = a_vss + dsa * a_dV[2];
    a_vsa = a_vsa - dsa * a_dV[2];
    a_wss = a_wss + dsa * a_dV[3];
    a_wsa = a_wsa - dsa * a_dV[3];
    a_ess = a_ess + a_dV[4];
    a_esa = a_esa - a_dV[4];
    a_byss = a_byss + a_dV[5];
    a_bysa = a_bysa - a_dV[5];
    a_bzss = a_bzss + a_dV[6];
    a_bzsa = a_bzsa - a_dV[6];
    // dU
    a_dsa = a_dsa + a_dU[0] + a_dU[1] * sM + a_dU[2] * vsa + a_dU[3] * wsa;
    aXd = aXd - a_dU[0] - a_dU[2] * X.v - a_dU[3] * X.w;
    a_sM = a_sM + a_dU[1] * dsa;
    a_mu = a_mu - a_dU[1];
    a_vsa = a_vsa + a_dU[2] * dsa;
    aXv = aXv - a_dU[2] * X.d;
    a_wsa = a_wsa + a_dU[3] * dsa;
    aXw = aXw - a_dU[3] * X.d;
    a_esa = a_esa + a_dU[4];
    a_eX = a_eX - a_dU[4];
    a_bysa = a_bysa + a_dU[5];
    aXby = aXby - a_dU[5];
    a_bzsa = a_bzsa + a_dU[6];
    aXbz = aXbz - a_dU[6];
    // physical flux of X
    {
        const double aF0 = a_f[0], aF1 = a_f[1], aF2 = a_f[2], aF3 = a_f[3], aF4 = a_f[4];
        const double aF5 = a_f[5], aF6 = a_f[6];
        a_mu = a_mu + aF0 + aF1 * X.u + aF2 * X.v + aF3 * X.w;
        aXu = aXu + aF1 * mu + aF4 * (e + pt) + aF5 * X.by + aF6 * X.bz;
        a_ptX = a_ptX + aF1 + aF4 * X.u;
        a_bn2 = a_bn2 - aF1;
        aXv = aXv + aF2 * mu - aF5 * bn;
        aXw = aXw + aF3 * mu - aF6 * bn;
        a_bn = a_bn - aF2 * X.by - aF3 * X.bz - aF4 * vbX - aF5 * X.v - aF6 * X.w;
        aXby = aXby - aF2 * bn + aF5 * X.u;
        aXbz = aXbz - aF3 * bn + aF6 * X.u;
        a_eX = a_eX + aF4 * X.u;
        const double a_vbX = -aF4 * bn;
        aXu = aXu + a_vbX * bn;
        a_bn = a_bn + a_vbX * X.u;
        aXv = aXv + a_vbX * X.by;
        aXby = aXby + a_vbX * X.v;
        aXw = aXw + a_vbX * X.bz;
        aXbz = aXbz + a_vbX * X.w;
        aXd = aXd + a_mu * X.u;
        aXu = aXu + a_mu * X.d;
    }
    // chosen-side star quantities back to their side
    if (left) {
        a_ds[0] = a_ds[0] + a_dsa; a_vs[0] = a_vs[0] + a_vsa; a_ws[0] = a_ws[0] + a_wsa;
        a_es[0] = a_es[0] + a_esa; a_bys[0] = a_bys[0] + a_bysa; a_bzs[0] = a_bzs[0] + a_bzsa;
    } else {
        a_ds[1] = a_ds[1] + a_dsa; a_vs[1] = a_vs[1] + a_vsa; a_ws[1] = a_ws[1] + a_wsa;
        a_es[1] = a_es[1] + a_esa; a_bys[1] = a_bys[1] + a_bysa; a_bzs[1] = a_bzs[1] + a_bzsa;
    }
    // ess
    double a_vbss = 0.0;
    if (left) {
        a_es[0] = a_es[0] + a_ess;
        a_rL = a_rL - a_ess * sg * (vbs[0] - vbss);
        a_vbs[0] = a_vbs[0] - a_ess * r * sg;
        a_vbss = a_vbss + a_ess * r * sg;
    } else {
        a_es[1] = a_es[1] + a_ess;
        a_rR = a_rR + a_ess * sg * (vbs[1] - vbss);
        a_vbs[1] = a_vbs[1] + a_ess * r * sg;
        a_vbss = a_vbss - a_ess * r * sg;
    }
    (void)vbs_a;
    // ss
    a_sM = a_sM + a_ss;
    if (left) {
        a_bn = a_bn - a_ss * abs_slope(bn) * irL;
        a_rL = a_rL + a_ss * fabs(bn) * (irL * irL);
    } else {
        a_bn = a_bn + a_ss * abs_slope(bn) * irR;
        a_rR = a_rR - a_ss * fabs(bn) * (irR * irR);
    }
    // vbss
    a_sM = a_sM + a_vbss * bn;
    a_bn = a_bn + a_vbss * sM;
    a_vss = a_vss + a_vbss * byss;
    a_byss = a_byss + a_vbss * vss;
    a_wss = a_wss + a_vbss * bzss;
    a_bzss = a_bzss + a_vbss * wss;
    // double-star states
    {
        const double a_nv = a_vss * isum, a_nw = a_wss * isum;
        const double a_nby = a_byss * isum, a_nbz = a_bzss * isum;
        const double a_isum = a_vss * nv + a_wss * nw + a_byss * nby + a_bzss * nbz;
        const double dvs = vs[1] - vs[0], dws = ws[1] - ws[0];
        a_rL = a_rL + a_nv * vs[0] + a_nw * ws[0] + a_nby * (bys[1] + sg * rR * dvs)
               + a_nbz * (bzs[1] + sg * rR * dws);
        a_rR = a_rR + a_nv * vs[1] + a_nw * ws[1] + a_nby * (bys[0] + sg * rL * dvs)
               + a_nbz * (bzs[0] + sg * rL * dws);
        a_vs[0] = a_vs[0] + a_nv * rL - a_nby * sg * rL * rR;
        a_vs[1] = a_vs[1] + a_nv * rR + a_nby * sg * rL * rR;
        a_ws[0] = a_ws[0] + a_nw * rL - a_nbz * sg * rL * rR;
        a_ws[1] = a_ws[1] + a_nw * rR + a_nbz * sg * rL * rR;
        a_bys[1] = a_bys[1] + a_nv * sg + a_nby * rL;
        a_bys[0] = a_bys[0] - a_nv * sg + a_nby * rR;
        a_bzs[1] = a_bzs[1] + a_nw * sg + a_nbz * rL;
        a_bzs[0] = a_bzs[0] - a_nw * sg + a_nbz * rR;
        const double a_rsum = -a_isum * isum * isum;
        a_rL = a_rL + a_rsum;
        a_rR = a_rR + a_rsum;
        a_ds[0] = a_ds[0] + a_rL * (0.5 * irL);
        a_ds[1] = a_ds[1] + a_rR * (0.5 * irR);
    }
    // single-star states of both sides
    double aLs[7] = {0, 0, 0, 0, 0, 0, 0}, aRs[7] = {0, 0, 0, 0, 0, 0, 0};  // d u v w (p unused) by bz
    double a_S2[2] = {0.0, 0.0}, a_pt2[2] = {0.0, 0.0}, a_e2[2] = {0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const W7 &Y = a == 0 ? L : R;
        const double pty = a == 0 ? ptL : ptR;
        const double ey = a == 0 ? eL : eR;
        double *aY = a == 0 ? aLs : aRs;
        double a_num_e = a_es[a] * issm[a];
        double a_issm = a_es[a] * num_e[a];
        double a_su = a_num_e * ey;
        a_e2[a] = a_e2[a] + a_num_e * su[a];
        a_pt2[a] = a_pt2[a] - a_num_e * Y.u;
        aY[1] = aY[1] - a_num_e * pty;
        a_pts = a_pts + a_num_e * sM;
        a_sM = a_sM + a_num_e * pts;
        a_bn = a_bn + a_num_e * (vb[a] - vbs[a]);
        const double a_vb = a_num_e * bn;
        a_vbs[a] = a_vbs[a] - a_num_e * bn;
        // vb = u bn + v by + w bz
        aY[1] = aY[1] + a_vb * bn;
        a_bn = a_bn + a_vb * Y.u;
        aY[2] = aY[2] + a_vb * Y.by;
        aY[5] = aY[5] + a_vb * Y.v;
        aY[3] = aY[3] + a_vb * Y.bz;
        aY[6] = aY[6] + a_vb * Y.w;
        // vbs = sM bn + vs bys + ws bzs
        a_sM = a_sM + a_vbs[a] * bn;
        a_bn = a_bn + a_vbs[a] * sM;
        a_vs[a] = a_vs[a] + a_vbs[a] * bys[a];
        a_bys[a] = a_bys[a] + a_vbs[a] * vs[a];
        a_ws[a] = a_ws[a] + a_vbs[a] * bzs[a];
        a_bzs[a] = a_bzs[a] + a_vbs[a] * ws[a];
        // bys = by t2, bzs = bz t2, vs = v - by t1, ws = w - bz t1
        aY[5] = aY[5] + a_bys[a] * t2[a] - a_vs[a] * t1[a];
        aY[6] = aY[6] + a_bzs[a] * t2[a] - a_ws[a] * t1[a];
        const double a_t2 = a_bys[a] * Y.by + a_bzs[a] * Y.bz;
        const double a_t1 = -a_vs[a] * Y.by - a_ws[a] * Y.bz;
        aY[2] = aY[2] + a_vs[a];
        aY[3] = aY[3] + a_ws[a];
        double a_den = 0.0;
        if (!degen[a]) {
            const double a_iden = a_t1 * bn * (sM - Y.u) + a_t2 * (Y.d * su[a] * su[a] - bn2);
            a_bn = a_bn + a_t1 * (sM - Y.u) * iden[a];
            a_sM = a_sM + a_t1 * bn * iden[a];
            aY[1] = aY[1] - a_t1 * bn * iden[a];
            aY[0] = aY[0] + a_t2 * su[a] * su[a] * iden[a];
            a_su = a_su + a_t2 * 2.0 * Y.d * su[a] * iden[a];
            a_bn2 = a_bn2 - a_t2 * iden[a];
            a_den = -a_iden * iden[a] * iden[a];
        }
        // den = d su ssm - bn^2
        aY[0] = aY[0] + a_den * su[a] * ssm[a];
        a_su = a_su + a_den * Y.d * ssm[a];
        double a_ssm = a_den * Y.d * su[a];
        a_bn2 = a_bn2 - a_den;
        // ds = d su issm
        aY[0] = aY[0] + a_ds[a] * su[a] * issm[a];
        a_su = a_su + a_ds[a] * Y.d * issm[a];
        a_issm = a_issm + a_ds[a] * Y.d * su[a];
        a_ssm = a_ssm - a_issm * issm[a] * issm[a];
        // ssm = S - sM, su = S - u
        a_S2[a] = a_S2[a] + a_ssm + a_su;
        a_sM = a_sM - a_ssm;
        aY[1] = aY[1] - a_su;
    }
    // the chosen side's own quantities
    if (left) { a_S2[0] = a_S2[0] + a_S; a_pt2[0] = a_pt2[0] + a_ptX; a_e2[0] = a_e2[0] + a_eX; }
    else { a_S2[1] = a_S2[1] + a_S; a_pt2[1] = a_pt2[1] + a_ptX; a_e2[1] = a_e2[1] + a_eX; }
    // pts, sM, iq
    double a_qL = 0.0, a_qR = 0.0, a_uL = 0.0, a_uR = 0.0;
    {
        const double a_np = a_pts * iq, a_nm = a_sM * iq;
        const double a_iq = a_pts * num_p + a_sM * num_m;
        a_qR = a_qR + a_np * (ptL + qL * (R.u - L.u)) + a_nm * R.u;
        a_qL = a_qL + a_np * (-ptR + qR * (R.u - L.u)) - a_nm * L.u;
        a_pt2[0] = a_pt2[0] + a_np * qR + a_nm;
        a_pt2[1] = a_pt2[1] - a_np * qL - a_nm;
        a_uR = a_uR + a_np * qL * qR + a_nm * qR;
        a_uL = a_uL - a_np * qL * qR - a_nm * qL;
        const double a_dq = -a_iq * iq * iq;
        a_qR = a_qR + a_dq;
        a_qL = a_qL - a_dq;
    }
    // qL = (sL - uL) dL, qR = (sR - uR) dR
    double a_dL = a_qL * (sL - L.u), a_dR = a_qR * (sR - R.u);
    a_S2[0] = a_S2[0] + a_qL * L.d;
    a_uL = a_uL - a_qL * L.d;
    a_S2[1] = a_S2[1] + a_qR * R.d;
    a_uR = a_uR - a_qR * R.d;
    // sL = min(uL, uR) - cmax, sR = max(uL, uR) + cmax
    if (uminR) a_uR = a_uR + a_S2[0]; else a_uL = a_uL + a_S2[0];
    if (umaxR) a_uR = a_uR + a_S2[1]; else a_uL = a_uL + a_S2[1];
    const double a_cmax = a_S2[1] - a_S2[0];
    // e = p / (g - 1) + rho u^2 / 2 + pb, pt = p + pb, pb = (bn^2 + by^2 + bz^2) / 2
    double a_pL = a_pt2[0] + a_e2[0] * gm1i, a_pR = a_pt2[1] + a_e2[1] * gm1i;
    const double a_pbL = a_pt2[0] + a_e2[0], a_pbR = a_pt2[1] + a_e2[1];
    a_dL = a_dL + 0.5 * u2L * a_e2[0];
    a_dR = a_dR + 0.5 * u2R * a_e2[1];
    a_uL = a_uL + L.d * L.u * a_e2[0];
    a_uR = a_uR + R.d * R.u * a_e2[1];
    double a_vL = L.d * L.v * a_e2[0], a_wL = L.d * L.w * a_e2[0];
    double a_vR = R.d * R.v * a_e2[1], a_wR = R.d * R.w * a_e2[1];
    double a_byL = L.by * a_pbL, a_bzL = L.bz * a_pbL;
    double a_byR = R.by * a_pbR, a_bzR = R.bz * a_pbR;
    a_bn2 = a_bn2 + 0.5 * (a_pbL + a_pbR);
    // fast speeds: only the larger one (c_max) has a cotangent; its forward
    // terms are evaluated again here rather than kept alive through the
    // reverse.  d c_f / d cf2 = 1 / (2 c_f) = rho rq, 1 / (2 rho) = cf2 / num
    {
        const W7 &Xc = cmaxR ? R : L;
        FastSq q;
        double rq;
        fast_fwd(Xc, q, rq);
        const double i2d = (q.gp + q.b2 + q.disc) * rq * rq;
        const double idc = q.disc > 0.0 ? 1.0 / q.disc : 0.0;
        double a_d = 0.0, a_p = 0.0, a_by = 0.0, a_bz = 0.0;
        fast_sq_rev(q, i2d, idc, bn, Xc.by, Xc.bz, gam, a_cmax * (Xc.d * rq), 0.0, a_d, a_p, a_bn,
                    a_by, a_bz);
        if (cmaxR) {
            a_dR = a_dR + a_d; a_pR = a_pR + a_p; a_byR = a_byR + a_by; a_bzR = a_bzR + a_bz;
        } else {
            a_dL = a_dL + a_d; a_pL = a_pL + a_p; a_byL = a_byL + a_by; a_bzL = a_bzL + a_bz;
        }
    }
    a_bn = a_bn + 2.0 * bn * a_bn2;

    // chosen-side state cotangents
    const double sx = left ? 1.0 : 0.0, sy = 1.0 - sx;
    aL.d = aL.d + a_dL + aLs[0] + sx * aXd;
    aL.u = aL.u + a_uL + aLs[1] + sx * aXu;
    aL.v = aL.v + a_vL + aLs[2] + sx * aXv;
    aL.w = aL.w + a_wL + aLs[3] + sx * aXw;
    aL.p = aL.p + a_pL;
    aL.by = aL.by + a_byL + aLs[5] + sx * aXby;
    aL.bz = aL.bz + a_bzL + aLs[6] + sx * aXbz;
    aR.d = aR.d + a_dR + aRs[0] + sy * aXd;
    aR.u = aR.u + a_uR + aRs[1] + sy * aXu;
    aR.v = aR.v + a_vR + aRs[2] + sy * aXv;
    aR.w = aR.w + a_wR + aRs[3] + sy * aXw;
    aR.p = aR.p + a_pR;
    aR.by = aR.by + a_byR + aRs[5] + sy * aXby;
    aR.bz = aR.bz + a_bzR + aRs[6] + sy * aXbz;
    a_bn_out = a_bn_out + a_bn;
}

// ---------------------------------------------------------------------------
// eigen-system reverse
// ---------------------------------------------------------------------------
struct EigenA {  // cotangents of the Eigen fields used by project / unproject
    double d, sqd, asq, a, ia2, cf, cs, af, as, by, bz, nf, ns, qf, qs, pf, ps, bf, bs, sr;
};

VLCT_DEV void eigen_zero(EigenA &A)
{
    A.d = 0.0; A.sqd = 0.0; A.asq = 0.0; A.a = 0.0; A.ia2 = 0.0; A.cf = 0.0; A.cs = 0.0;
    A.af = 0.0; A.as = 0.0; A.by = 0.0; A.bz = 0.0; A.nf = 0.0; A.ns = 0.0; A.qf = 0.0;
    A.qs = 0.0; A.pf = 0.0; A.ps = 0.0; A.bf = 0.0; A.bs = 0.0; A.sr = 0.0;
}

// (a_c, a_bn) += (d E / d(c, bn))^T A for eigen_setup(c, bn, gam)
VLCT_DEV void eigen_rev(const W7 &c, double bn_in, double gam, const EigenA &A, W7 &a_c,
                        double &a_bn_in)
{
    // forward (the formulas of eigen_setup)
    const double gp = gam * c.p;
    const double tiny2 =
        kBperpTiny * kBperpTiny * (gp + bn_in * bn_in + c.by * c.by + c.bz * c.bz);
    const bool snap_n = bn_in * bn_in <= tiny2;
    const bool snap_1 = c.by * c.by <= tiny2;
    const bool snap_2 = c.bz * c.bz <= tiny2;
    const double bn = snap_n ? 0.0 : bn_in;
    const double bt1 = snap_1 ? 0.0 : c.by;
    const double bt2 = snap_2 ? 0.0 : c.bz;
    // r = 1/sqrt(rho), q = 1/sqrt(gP)
    const double r = mrsqrt(c.d), q = mrsqrt(gp);
    const double id = r * r;
    const double sqd = c.d * r;
    const double asq = gp * id;
    const double a = gp * q * r;
    const double ia = sqd * q;  // 1 / a
    const double ia2 = c.d * q * q;
    FastSq fq = fast_sq_terms(c.p, bn * bn, bt1, bt2, gam);
    const double bp2 = fq.bp2, disc = fq.disc;
    const double cf2 = (gp + bn * bn + bp2 + disc) * (0.5 * id);
    fq.cf2 = cf2;
    const double cf = msqrt(cf2);
    const double icf = 1.0 / cf;
    const double kcs = a * r * icf;  // c_s / |B_n|
    const double cs = kcs * fabs(bn);
    const bool haveperp = bp2 > tiny2;
    const double ibp = mrsqrt(haveperp ? bp2 : 1.0);
    const double tdiff = fq.t;
    const bool split = disc > kCfCsTiny * c.d * cf2;
    const double idisc = 0.5 / disc;
    const double qfv = (disc + tdiff) * idisc, qsv = (disc - tdiff) * idisc;
    const double af2 = fmin(fmax(qfv, 0.0), 1.0);
    const double as2 = fmin(fmax(qsv, 0.0), 1.0);
    const double af = split ? msqrt(af2) : 1.0;
    const double as = split ? msqrt(as2) : 0.0;
    const double s = bn >= 0.0 ? 1.0 : -1.0;
    // 1 / sqrt(rho) = r and 1 / (a sqrt(rho)) = q

    // reverse
    double a_isqd = 0.5 * s * A.sr;
    double a_af = A.af - 0.5 * q * A.bs;
    double a_as = A.as + 0.5 * q * A.bf;
    const double a_iasq = -0.5 * af * A.bs + 0.5 * as * A.bf;
    a_isqd = a_isqd + a_iasq * ia;
    double a_a = A.a - a_iasq * q * ia;
    double a_sqd = A.sqd - a_isqd * id;
    double a_ia2 = A.ia2;
    double a_id = 0.0;
    a_as = a_as + 0.5 * ia2 * id * A.ps;
    a_ia2 = a_ia2 + 0.5 * as * id * A.ps;
    a_id = a_id + 0.5 * as * ia2 * A.ps;
    a_af = a_af + 0.5 * ia2 * id * A.pf;
    a_ia2 = a_ia2 + 0.5 * af * id * A.pf;
    a_id = a_id + 0.5 * af * ia2 * A.pf;
    double a_cf = A.cf, a_cs = A.cs;
    a_af = a_af + 0.5 * s * cf * ia2 * A.qs + 0.5 * cf * ia2 * A.nf;
    a_cf = a_cf + 0.5 * s * af * ia2 * A.qs + 0.5 * af * ia2 * A.nf;
    a_ia2 = a_ia2 + 0.5 * s * af * cf * A.qs + 0.5 * af * cf * A.nf;
    a_as = a_as + 0.5 * s * cs * ia2 * A.qf + 0.5 * cs * ia2 * A.ns;
    a_cs = a_cs + 0.5 * s * as * ia2 * A.qf + 0.5 * as * ia2 * A.ns;
    a_ia2 = a_ia2 + 0.5 * s * as * cs * A.qf + 0.5 * as * cs * A.ns;
    // alpha_f, alpha_s
    double a_disc = 0.0, a_tdiff = 0.0;
    if (split) {
        const double a_af2 = a_af * sqrt_slope(af);
        const double a_as2 = a_as * sqrt_slope(as);
        // the clamps pass their argument through on [0, 1]
        const double a_qf = (qfv >= 0.0 && qfv <= 1.0) ? a_af2 : 0.0;
        const double a_qs = (qsv >= 0.0 && qsv <= 1.0) ? a_as2 : 0.0;
        const double a_idisc = (disc + tdiff) * a_qf + (disc - tdiff) * a_qs;
        a_disc = idisc * (a_qf + a_qs) - a_idisc * (2.0 * idisc * idisc);
        a_tdiff = idisc * (a_qf - a_qs);
    }
    double a_d = A.d, a_p = gam * a_tdiff, a_bn = -2.0 * bn * a_tdiff;
    double a_bt1 = -2.0 * bt1 * a_tdiff, a_bt2 = -2.0 * bt2 * a_tdiff;
    // beta_t1, beta_t2 = bt / sqrt(bp2)
    if (haveperp) {
        a_bt1 = a_bt1 + ibp * A.by;
        a_bt2 = a_bt2 + ibp * A.bz;
        const double a_ibp = bt1 * A.by + bt2 * A.bz;
        const double a_bp = -a_ibp * ibp * ibp;
        a_bt1 = a_bt1 + bt1 * ibp * a_bp;
        a_bt2 = a_bt2 + bt2 * ibp * a_bp;
    }
    // slow and fast speeds: c_s^2 = a^2 B_n^2 / (rho c_f^2), so with
    // h = c_s a_cs / 2 the slow speed sends h / a^2 to a^2, h rho to 1/rho and
    // -h / c_f^2 to c_f^2, and c_s / B_n to B_n
    const double h = 0.5 * a_cs * cs;
    double a_cf2 = a_cf * (0.5 * icf);
    double a_asq = h * ia2;
    a_bn = a_bn + a_cs * kcs * s;
    a_id = a_id + h * c.d;
    a_cf2 = a_cf2 - h * (icf * icf);
    fast_sq_rev(fq, 0.5 * id, 2.0 * idisc, bn, bt1, bt2, gam, a_cf2, a_disc, a_d, a_p, a_bn,
                a_bt1, a_bt2);
    // sound speed, rho^(1/2), 1/a^2 = rho / (gP)
    a_d = a_d + a_ia2 * (q * q);
    double a_gp = -a_ia2 * ia2 * (q * q);
    a_asq = a_asq + A.asq + a_a * (0.5 * ia);
    a_gp = a_gp + id * a_asq;
    a_id = a_id + gp * a_asq;
    a_d = a_d + a_sqd * (0.5 * r);
    a_p = a_p + gam * a_gp;
    a_d = a_d - a_id * id * id;
    a_c.d = a_c.d + a_d;
    a_c.p = a_c.p + a_p;
    if (!snap_1) a_c.by = a_c.by + a_bt1;
    if (!snap_2) a_c.bz = a_c.bz + a_bt2;
    if (!snap_n) a_bn_in = a_bn_in + a_bn;
}

// a_dw += L^T a_a for a = project(E, dw), and A += d(a_a . L dw)/dE
VLCT_DEV void project_rev(const Eigen &E, const double dw[7], const double aa[7], double adw[7],
                          EigenA &A)
{
    const double vpar = E.by * dw[2] + E.bz * dw[3];
    const double vperp = -E.bz * dw[2] + E.by * dw[3];
    const double bpar = E.by * dw[5] + E.bz * dw[6];
    const double bperp = -E.bz * dw[5] + E.by * dw[6];
    const double a_hf = aa[0] + aa[6], a_gf = aa[6] - aa[0];
    const double a_hs = aa[2] + aa[4], a_gs = aa[4] - aa[2];
    const double a_vperp = 0.5 * (aa[1] + aa[5]);
    const double a_bperp = E.sr * (aa[1] - aa[5]);
    A.sr = A.sr + bperp * (aa[1] - aa[5]);
    adw[0] = adw[0] + aa[3];
    adw[4] = adw[4] - E.ia2 * aa[3] + E.pf * a_hf + E.ps * a_hs;
    A.ia2 = A.ia2 - dw[4] * aa[3];
    A.pf = A.pf + dw[4] * a_hf;
    A.bf = A.bf + bpar * a_hf;
    A.ps = A.ps + dw[4] * a_hs;
    A.bs = A.bs + bpar * a_hs;
    const double a_bpar = E.bf * a_hf + E.bs * a_hs;
    A.nf = A.nf + dw[1] * a_gf;
    A.qf = A.qf - vpar * a_gf;
    A.ns = A.ns + dw[1] * a_gs;
    A.qs = A.qs + vpar * a_gs;
    adw[1] = adw[1] + E.nf * a_gf + E.ns * a_gs;
    const double a_vpar = -E.qf * a_gf + E.qs * a_gs;
    A.by = A.by + dw[2] * a_vpar + dw[3] * a_vperp + dw[5] * a_bpar + dw[6] * a_bperp;
    A.bz = A.bz + dw[3] * a_vpar - dw[2] * a_vperp + dw[6] * a_bpar - dw[5] * a_bperp;
    adw[2] = adw[2] + E.by * a_vpar - E.bz * a_vperp;
    adw[3] = adw[3] + E.bz * a_vpar + E.by * a_vperp;
    adw[5] = adw[5] + E.by * a_bpar - E.bz * a_bperp;
    adw[6] = adw[6] + E.bz * a_bpar + E.by * a_bperp;
}

// a_a += R^T a_dw for dw = unproject(E, a), and A += d(a_dw . R a)/dE
VLCT_DEV void unproject_rev(const Eigen &E, const double a[7], const double adw[7], double aa[7],
                            EigenA &A)
{
    const double fsum = a[0] + a[6], fdif = a[6] - a[0];
    const double ssum = a[2] + a[4], sdif = a[4] - a[2];
    const double asum = a[1] + a[5], adif = a[5] - a[1];
    const double tpar = -E.s * (E.as * E.cs * fdif - E.af * E.cf * sdif);
    const double H = E.as * fsum - E.af * ssum;
    const double bmag = E.a * E.sqd * H;
    const double sb = E.s * E.sqd * adif;
    const double G = E.af * fsum + E.as * ssum;
    const double a_G = E.d * adw[0] + E.d * E.asq * adw[4];
    A.d = A.d + G * adw[0] + E.asq * G * adw[4];
    A.asq = A.asq + E.d * G * adw[4];
    aa[3] = aa[3] + adw[0];
    double a_fsum = a_G * E.af, a_ssum = a_G * E.as;
    A.af = A.af + a_G * fsum + adw[1] * E.cf * fdif;
    A.as = A.as + a_G * ssum + adw[1] * E.cs * sdif;
    A.cf = A.cf + adw[1] * E.af * fdif;
    A.cs = A.cs + adw[1] * E.as * sdif;
    double a_fdif = adw[1] * E.af * E.cf, a_sdif = adw[1] * E.as * E.cs;
    A.by = A.by + adw[2] * tpar + adw[3] * asum + adw[5] * bmag - adw[6] * sb;
    A.bz = A.bz - adw[2] * asum + adw[3] * tpar + adw[5] * sb + adw[6] * bmag;
    const double a_tpar = adw[2] * E.by + adw[3] * E.bz;
    double a_asum = -adw[2] * E.bz + adw[3] * E.by;
    const double a_bmag = adw[5] * E.by + adw[6] * E.bz;
    const double a_sb = adw[5] * E.bz - adw[6] * E.by;
    // tpar
    A.as = A.as - E.s * E.cs * fdif * a_tpar;
    A.cs = A.cs - E.s * E.as * fdif * a_tpar;
    a_fdif = a_fdif - E.s * E.as * E.cs * a_tpar;
    A.af = A.af + E.s * E.cf * sdif * a_tpar;
    A.cf = A.cf + E.s * E.af * sdif * a_tpar;
    a_sdif = a_sdif + E.s * E.af * E.cf * a_tpar;
    // bmag
    A.a = A.a + E.sqd * H * a_bmag;
    A.sqd = A.sqd + E.a * H * a_bmag + E.s * adif * a_sb;
    const double a_H = E.a * E.sqd * a_bmag;
    A.as = A.as + fsum * a_H;
    A.af = A.af - ssum * a_H;
    a_fsum = a_fsum + E.as * a_H;
    a_ssum = a_ssum - E.af * a_H;
    const double a_adif = E.s * E.sqd * a_sb;
    aa[0] = aa[0] + a_fsum - a_fdif;
    aa[6] = aa[6] + a_fsum + a_fdif;
    aa[2] = aa[2] + a_ssum - a_sdif;
    aa[4] = aa[4] + a_ssum + a_sdif;
    aa[1] = aa[1] + a_asum - a_adif;
    aa[5] = aa[5] + a_asum + a_adif;
}

// ---------------------------------------------------------------------------
// PLMC / PLMP reverse: given the cotangents of the interface states (after
// their floors: a floored component carries none), add those of the three
// stencil states and of the cell's normal field
// ---------------------------------------------------------------------------
template <bool CHAR>
VLCT_DEV void plmc_rev(const W7 &wm, const W7 &w0, const W7 &wp, double bn, double gam,
                       const double a_fm[7], const double a_fp[7], W7 &a_wm, W7 &a_w0, W7 &a_wp,
                       double &a_bn)
{
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
    // limiter (the fmin order of plmc): which difference the limited slope
    // took (0: left, 1: right, 2: centred, 3: van Leer) and its slope there
    int pick[7];
    double coef[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        const double A2l = 2.0 * fabs(al[m]), A2r = 2.0 * fabs(ar[m]);
        const double Ac = fabs(ac[m]), Av = fabs(av[m]);
        const bool lr_r = takes_second_min(A2l, A2r);
        const double mlr = lr_r ? A2r : A2l;
        const bool cv_v = takes_second_min(Ac, Av);
        const double mcv = cv_v ? Av : Ac;
        const bool pick_cv = takes_second_min(mlr, mcv);
        const double lim = pick_cv ? mcv : mlr;
        const bool on = al[m] * ar[m] > 0.0;
        const double sgn = copysign(1.0, ac[m]);  // the sign copysign gives lim
        am[m] = on ? sgn * lim : 0.0;
        const double g = on ? sgn : 0.0;
        pick[m] = pick_cv ? (cv_v ? 3 : 2) : (lr_r ? 1 : 0);
        const double x = pick_cv ? (cv_v ? av[m] : ac[m]) : (lr_r ? ar[m] : al[m]);
        coef[m] = g * (pick_cv ? 1.0 : 2.0) * abs_slope(x);
    }
    // fp = x0 + dw / 2, fm = x0 - dw / 2
    double adw[7], ax0[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        adw[c] = 0.5 * (a_fp[c] - a_fm[c]);
        ax0[c] = a_fp[c] + a_fm[c];
    }
    double aam[7] = {0, 0, 0, 0, 0, 0, 0};
    EigenA EA;
    if (CHAR) {
        eigen_zero(EA);
        unproject_rev(E, am, adw, aam, EA);
    } else {
#pragma unroll
        for (int c = 0; c < 7; ++c) aam[c] = adw[c];
    }
    double aal[7], aar[7], aac[7], aav[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        const double v = coef[m] * aam[m];
        aal[m] = pick[m] == 0 ? v : 0.0;
        aar[m] = pick[m] == 1 ? v : 0.0;
        aac[m] = pick[m] == 2 ? v : 0.0;
        aav[m] = pick[m] == 3 ? v : 0.0;
    }
    double adl[7] = {0, 0, 0, 0, 0, 0, 0}, adr[7] = {0, 0, 0, 0, 0, 0, 0};
    double adc[7] = {0, 0, 0, 0, 0, 0, 0}, adv[7] = {0, 0, 0, 0, 0, 0, 0};
    if (CHAR) {
        project_rev(E, dl, aal, adl, EA);
        project_rev(E, dr, aar, adr, EA);
        project_rev(E, dc, aac, adc, EA);
        project_rev(E, dv, aav, adv, EA);
    } else {
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            adl[c] = aal[c];
            adr[c] = aar[c];
            adc[c] = aac[c];
            adv[c] = aav[c];
        }
    }
    // van Leer difference, then the stencil differences
    double am_[7], ap_[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        const double pr = dl[c] * dr[c];
        if (pr > 0.0) {
            const double s = dl[c] + dr[c];
            const double is2 = 1.0 / (s * s);
            adl[c] = adl[c] + adv[c] * 2.0 * dr[c] * dr[c] * is2;
            adr[c] = adr[c] + adv[c] * 2.0 * dl[c] * dl[c] * is2;
        }
        ax0[c] = ax0[c] + adl[c] - adr[c];
        am_[c] = -adl[c] - 0.5 * adc[c];
        ap_[c] = adr[c] + 0.5 * adc[c];
    }
    W7 ae0{ax0[0], ax0[1], ax0[2], ax0[3], ax0[4], ax0[5], ax0[6]};
    if (CHAR) eigen_rev(w0, bn, gam, EA, ae0, a_bn);
    a_w0.d = a_w0.d + ae0.d; a_w0.u = a_w0.u + ae0.u; a_w0.v = a_w0.v + ae0.v;
    a_w0.w = a_w0.w + ae0.w; a_w0.p = a_w0.p + ae0.p; a_w0.by = a_w0.by + ae0.by;
    a_w0.bz = a_w0.bz + ae0.bz;
    a_wm.d = a_wm.d + am_[0]; a_wm.u = a_wm.u + am_[1]; a_wm.v = a_wm.v + am_[2];
    a_wm.w = a_wm.w + am_[3]; a_wm.p = a_wm.p + am_[4]; a_wm.by = a_wm.by + am_[5];
    a_wm.bz = a_wm.bz + am_[6];
    a_wp.d = a_wp.d + ap_[0]; a_wp.u = a_wp.u + ap_[1]; a_wp.v = a_wp.v + ap_[2];
    a_wp.w = a_wp.w + ap_[3]; a_wp.p = a_wp.p + ap_[4]; a_wp.by = a_wp.by + ap_[5];
    a_wp.bz = a_wp.bz + ap_[6];
}

// ---------------------------------------------------------------------------
// PPMC / PPMP reverse
// ---------------------------------------------------------------------------
// ppm_face(am, a0, ap, app) reversed: adds the cotangents of its four inputs
// given that of its output
VLCT_DEV void ppm_face_rev(double am, double a0, double ap, double app, double af, double &a_am,
                           double &a_a0, double &a_ap, double &a_app)
{
    const double f0 = (7.0 / 12.0) * (a0 + ap) - (1.0 / 12.0) * (am + app);
    double a_f0 = 0.0;
    if ((f0 - a0) * (ap - f0) < 0.0) {
        // f = (a0 + ap) / 2 - lim / 6
        const double d2 = 3.0 * (a0 - 2.0 * f0 + ap);
        const double d2l = am - 2.0 * a0 + ap;
        const double d2r = a0 - 2.0 * ap + app;
        a_a0 = a_a0 + 0.5 * af;
        a_ap = a_ap + 0.5 * af;
        const double a_lim = -af / 6.0;
        if (d2 * d2l > 0.0 && d2 * d2r > 0.0) {
            // lim = sign(d2) min(C |d2l|, C |d2r|, |d2|): all three share d2's sign
            const double A = kPpmC * fabs(d2l), Bv = kPpmC * fabs(d2r), Cv = fabs(d2);
            const bool ab_b = takes_second_min(A, Bv);
            const double mab = ab_b ? Bv : A;
            const bool pick_c = takes_second_min(mab, Cv);
            if (pick_c) {
                const double a_d2 = a_lim;  // lim = d2
                a_a0 = a_a0 + 3.0 * a_d2;
                a_ap = a_ap + 3.0 * a_d2;
                a_f0 = a_f0 - 6.0 * a_d2;
            } else if (ab_b) {
                const double a_d2r = kPpmC * a_lim;  // lim = C d2r
                a_a0 = a_a0 + a_d2r;
                a_ap = a_ap - 2.0 * a_d2r;
                a_app = a_app + a_d2r;
            } else {
                const double a_d2l = kPpmC * a_lim;  // lim = C d2l
                a_am = a_am + a_d2l;
                a_a0 = a_a0 - 2.0 * a_d2l;
                a_ap = a_ap + a_d2l;
            }
        }
    } else {
        a_f0 = af;
    }
    a_a0 = a_a0 + (7.0 / 12.0) * a_f0;
    a_ap = a_ap + (7.0 / 12.0) * a_f0;
    a_am = a_am - (1.0 / 12.0) * a_f0;
    a_app = a_app - (1.0 / 12.0) * a_f0;
}

// the clamp fmax(fmin(lo_a, lo_b), fmin(v, fmax(hi_a, hi_b))) as ppmc writes it
// (bounds from the pair (0 or x0, neighbour)): returns which argument it
// passes through -- 0: v, 1: the first bound argument (0 / x0), 2: the
// neighbour
VLCT_DEV int clamp_pick(double x0, double nb, double v)
{
    const bool lo_nb = takes_second_min(x0, nb);
    const double lo = lo_nb ? nb : x0;
    const bool hi_nb = takes_second_max(x0, nb);
    const double hi = hi_nb ? nb : x0;
    const bool inner_hi = takes_second_min(v, hi);
    const double inner = inner_hi ? hi : v;
    const bool outer_inner = takes_second_max(lo, inner);
    if (outer_inner) return inner_hi ? (hi_nb ? 2 : 1) : 0;
    return lo_nb ? 2 : 1;
}

template <bool CHAR>
VLCT_DEV void ppmc_rev(const W7 &wmm, const W7 &wm, const W7 &w0, const W7 &wp, const W7 &wpp,
                       double bn, double gam, const double a_fm[7], const double a_fp[7],
                       W7 &a_wmm, W7 &a_wm, W7 &a_w0, W7 &a_wp, W7 &a_wpp, double &a_bn)
{
    // ---- forward (the steps of ppmc, the quantities the reverse needs kept)
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
    const double floor_c[7] = {0.0, fv, fv, fv, 0.0, fb, fb};
    double x0[7], xn[4][7], xs[4][7];
    to_arr(w0, x0);
    to_arr(wmm, xn[0]);
    to_arr(wm, xn[1]);
    to_arr(wp, xn[2]);
    to_arr(wpp, xn[3]);
    bool tie[4][7];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            const double d = xn[q][c] - x0[c];
            tie[q][c] = fabs(d) <= kPpmTie * (fabs(xn[q][c]) + fabs(x0[c]) + floor_c[c]);
            xs[q][c] = tie[q][c] ? 0.0 : d;
        }
    double a[4][7];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (CHAR) {
            project(E, xs[q], a[q]);
        } else {
#pragma unroll
            for (int c = 0; c < 7; ++c) a[q][c] = xs[q][c];
        }
    }
    double dplus[7], dminus[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        const double a_2 = a[0][m], a_1 = a[1][m], a1 = a[2][m], a2 = a[3][m];
        const double fl = ppm_face(a_2, a_1, 0.0, a1);
        const double fr = ppm_face(a_1, 0.0, a1, a2);
        double dp = fr, dm = -fl;
        if (dp * dm <= 0.0 || a1 * (-a_1) <= 0.0) {
            const double d2 = 6.0 * (fl + fr);
            const double d2c = a_1 + a1, d2l = a_2 - 2.0 * a_1, d2r = -2.0 * a1 + a2;
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

    // ---- reverse
    double a_x0[7] = {0, 0, 0, 0, 0, 0, 0}, a_xn[4][7];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 7; ++c) a_xn[q][c] = 0.0;
    double a_wpl[7], a_wmi[7];
    // primitive bounds and the CW84 constraints
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        const double xl = xn[1][c], xr = xn[2][c];
        const double up = x0[c] + wpl[c], um = x0[c] + wmi[c];
        const double vp = fmax(fmin(x0[c], xr), fmin(up, fmax(x0[c], xr)));
        const double vm = fmax(fmin(x0[c], xl), fmin(um, fmax(x0[c], xl)));
        const double tol = kPpmTie * (fabs(x0[c]) + fabs(xl) + fabs(xr) + floor_c[c]);
        double a_vp = a_fp[c], a_vm = a_fm[c];
        if (fabs(vp - up) > tol || fabs(vm - um) > tol) {
            const double dpp = vp - x0[c], dmm = x0[c] - vm;
            if (dpp * dmm <= 0.0) {
                // vp = vm = x0
                a_x0[c] = a_x0[c] + a_vp + a_vm;
                a_vp = 0.0;
                a_vm = 0.0;
            } else {
                double a_dpp = 0.0, a_dmm = 0.0;
                if (fabs(dpp) >= 2.0 * fabs(dmm)) {  // vp = x0 + 2 dmm
                    a_x0[c] = a_x0[c] + a_vp;
                    a_dmm = a_dmm + 2.0 * a_vp;
                    a_vp = 0.0;
                }
                if (fabs(dmm) >= 2.0 * fabs(dpp)) {  // vm = x0 - 2 dpp
                    a_x0[c] = a_x0[c] + a_vm;
                    a_dpp = a_dpp - 2.0 * a_vm;
                    a_vm = 0.0;
                }
                // dpp = vp - x0, dmm = x0 - vm (of the bounded values)
                a_vp = a_vp + a_dpp;
                a_x0[c] = a_x0[c] - a_dpp + a_dmm;
                a_vm = a_vm - a_dmm;
            }
        }
        // the bounds: each passes up / um, x0 or the neighbour through
        double a_up = 0.0, a_um = 0.0;
        const int pp = clamp_pick(x0[c], xr, up), pm = clamp_pick(x0[c], xl, um);
        if (pp == 0) a_up = a_vp; else if (pp == 1) a_x0[c] = a_x0[c] + a_vp; else a_xn[2][c] = a_xn[2][c] + a_vp;
        if (pm == 0) a_um = a_vm; else if (pm == 1) a_x0[c] = a_x0[c] + a_vm; else a_xn[1][c] = a_xn[1][c] + a_vm;
        a_x0[c] = a_x0[c] + a_up + a_um;
        a_wpl[c] = a_up;
        a_wmi[c] = a_um;
    }
    // back-projection
    double a_dplus[7] = {0, 0, 0, 0, 0, 0, 0}, a_dminus[7] = {0, 0, 0, 0, 0, 0, 0};
    EigenA EA;
    if (CHAR) {
        eigen_zero(EA);
        unproject_rev(E, dplus, a_wpl, a_dplus, EA);
        unproject_rev(E, dminus, a_wmi, a_dminus, EA);
    } else {
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            a_dplus[c] = a_wpl[c];
            a_dminus[c] = a_wmi[c];
        }
    }
    // per wave: the characteristic limiter chain
    double a_a[4][7];
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        const double a_2 = a[0][m], a_1 = a[1][m], a1 = a[2][m], a2 = a[3][m];
        const double fl = ppm_face(a_2, a_1, 0.0, a1);
        const double fr = ppm_face(a_1, 0.0, a1, a2);
        const double dp0 = fr, dm0 = -fl;
        double aa_2 = 0.0, aa_1 = 0.0, aa1 = 0.0, aa2 = 0.0;
        // recompute the limited dp, dm with their branch
        const bool ext = dp0 * dm0 <= 0.0 || a1 * (-a_1) <= 0.0;
        double dp = dp0, dm = dm0, ratio = 0.0, d2 = 0.0, lim = 0.0;
        int lim_pick = -1;  // 0: C d2l, 1: C d2r, 2: C d2c, 3: d2, -1: zero
        bool o1 = false, o2 = false;
        if (ext) {
            d2 = 6.0 * (fl + fr);
            const double d2c = a_1 + a1, d2l = a_2 - 2.0 * a_1, d2r = -2.0 * a1 + a2;
            if (d2 * d2c > 0.0 && d2 * d2l > 0.0 && d2 * d2r > 0.0) {
                const double L = kPpmC * fabs(d2l), R = kPpmC * fabs(d2r);
                const double Cc = kPpmC * fabs(d2c), Dd = fabs(d2);
                const bool lr = takes_second_min(L, R);
                const double mlr = lr ? R : L;
                const bool cd = takes_second_min(Cc, Dd);
                const double mcd = cd ? Dd : Cc;
                const bool pick2 = takes_second_min(mlr, mcd);
                lim_pick = pick2 ? (cd ? 3 : 2) : (lr ? 1 : 0);
                lim = copysign(pick2 ? mcd : mlr, d2);
            }
            ratio = d2 != 0.0 ? lim / d2 : 0.0;
            dp = dp0 * ratio;
            dm = dm0 * ratio;
        } else {
            o1 = fabs(dp0) >= 2.0 * fabs(dm0);
            if (o1) dp = 2.0 * dm0;
            o2 = fabs(dm0) >= 2.0 * fabs(dp);
            if (o2) dm = 2.0 * dp;
        }
        // dplus = clamp of dp to the pair (0, a1); dminus = clamp of -dm to (0, a_1)
        double a_dp = 0.0, a_dm = 0.0;
        {
            const int pk = clamp_pick(0.0, a1, dp);
            if (pk == 0) a_dp = a_dplus[m]; else if (pk == 2) aa1 = aa1 + a_dplus[m];
            const int mk = clamp_pick(0.0, a_1, -dm);
            if (mk == 0) a_dm = -a_dminus[m]; else if (mk == 2) aa_1 = aa_1 + a_dminus[m];
        }
        double a_fl = 0.0, a_fr = 0.0;
        if (ext) {
            const double a_dp0 = ratio * a_dp, a_dm0 = ratio * a_dm;
            const double a_ratio = dp0 * a_dp + dm0 * a_dm;
            double a_d2 = 0.0, a_lim = 0.0;
            if (d2 != 0.0) {
                a_lim = a_ratio / d2;
                a_d2 = -a_ratio * ratio / d2;
            }
            // lim = sign(d2) min(...): all candidates share d2's sign
            double a_d2l = 0.0, a_d2r = 0.0, a_d2c = 0.0;
            if (lim_pick == 0) a_d2l = kPpmC * a_lim;
            else if (lim_pick == 1) a_d2r = kPpmC * a_lim;
            else if (lim_pick == 2) a_d2c = kPpmC * a_lim;
            else if (lim_pick == 3) a_d2 = a_d2 + a_lim;
            a_fl = a_fl + 6.0 * a_d2 - a_dm0;
            a_fr = a_fr + 6.0 * a_d2 + a_dp0;
            aa_1 = aa_1 + a_d2c - 2.0 * a_d2l;
            aa1 = aa1 + a_d2c - 2.0 * a_d2r;
            aa_2 = aa_2 + a_d2l;
            aa2 = aa2 + a_d2r;
        } else {
            double a_dp1 = a_dp, a_dm0 = 0.0, a_dp0 = 0.0;
            if (o2) a_dp1 = a_dp1 + 2.0 * a_dm; else a_dm0 = a_dm0 + a_dm;
            if (o1) a_dm0 = a_dm0 + 2.0 * a_dp1; else a_dp0 = a_dp0 + a_dp1;
            a_fr = a_fr + a_dp0;
            a_fl = a_fl - a_dm0;
        }
        // fl = ppm_face(a_2, a_1, 0, a1), fr = ppm_face(a_1, 0, a1, a2)
        double dummy = 0.0;
        ppm_face_rev(a_2, a_1, 0.0, a1, a_fl, aa_2, aa_1, dummy, aa1);
        ppm_face_rev(a_1, 0.0, a1, a2, a_fr, aa_1, dummy, aa1, aa2);
        a_a[0][m] = aa_2;
        a_a[1][m] = aa_1;
        a_a[2][m] = aa1;
        a_a[3][m] = aa2;
    }
    // projections of the stencil differences, then the tie snapping
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double a_xs[7] = {0, 0, 0, 0, 0, 0, 0};
        if (CHAR) {
            project_rev(E, xs[q], a_a[q], a_xs, EA);
        } else {
#pragma unroll
            for (int c = 0; c < 7; ++c) a_xs[c] = a_a[q][c];
        }
#pragma unroll
        for (int c = 0; c < 7; ++c)
            if (!tie[q][c]) {
                a_xn[q][c] = a_xn[q][c] + a_xs[c];
                a_x0[c] = a_x0[c] - a_xs[c];
            }
    }
    W7 ae0{a_x0[0], a_x0[1], a_x0[2], a_x0[3], a_x0[4], a_x0[5], a_x0[6]};
    if (CHAR) eigen_rev(w0, bn, gam, EA, ae0, a_bn);
    W7 *outs[5] = {&a_wmm, &a_wm, &a_w0, &a_wp, &a_wpp};
    const double *src[5] = {a_xn[0], a_xn[1], nullptr, a_xn[2], a_xn[3]};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        W7 &o = *outs[q];
        if (q == 2) {
            o.d = o.d + ae0.d; o.u = o.u + ae0.u; o.v = o.v + ae0.v; o.w = o.w + ae0.w;
            o.p = o.p + ae0.p; o.by = o.by + ae0.by; o.bz = o.bz + ae0.bz;
        } else {
            const double *v = src[q];
            o.d = o.d + v[0]; o.u = o.u + v[1]; o.v = o.v + v[2]; o.w = o.w + v[3];
            o.p = o.p + v[4]; o.by = o.by + v[5]; o.bz = o.bz + v[6];
        }
    }
}

}  // namespace vlct
