// vlct_adjoint.hip -- adjoint (reverse derivative) of one VL+CT step (Caddy &
// Schneider, "Cholla-MHD", Sec. 2.2) on gfx950:
//
//   lam_in = (d U^{n+1} / d U^n)^T lam_out
//
// for a step of fixed size dt (dt is a parameter, not differentiated), with
// every branch (HLLD wave regions, limiter cases, CT upwind sides, floors)
// taken as in the forward evaluation at U^n.  The step is the composition
//   U^n -> W^n -> PCM/HLLD fluxes -> CT edge fields -> U^{n+1/2}
//       -> W^{n+1/2} -> reconstruction/HLLD fluxes -> CT edge fields -> U^{n+1};
// its transpose is applied stage by stage in reverse.  The linear parts (flux
// differences, curl, edge-field averaging with frozen upwind weights) are
// transposed by hand; the local non-linear maps (primitive recovery,
// -v x B, HLLD per face, reconstruction per cell) have their Jacobians formed
// by forward-mode dual numbers at the forward point, which follow the same
// branches as the double-precision code, and are applied transposed.
// Periodic boundaries; PCM, PLMC and PLMP correctors.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "vlct_common.hpp"

namespace vlct_ad {

// ---------------------------------------------------------------------------
// dual numbers: a value and kDir directional derivatives
// ---------------------------------------------------------------------------
constexpr int kDir = 8;

struct D8 {
    double v;
    double d[kDir];
    __host__ __device__ constexpr D8(double x = 0.0) : v(x), d{} {}
};

#define VLCT_AD_FN __host__ __device__ __forceinline__
VLCT_AD_FN D8 operator+(const D8 &a, const D8 &b)
{
    D8 r(a.v + b.v);
#pragma unroll
    for (int k = 0; k < kDir; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
VLCT_AD_FN D8 operator-(const D8 &a, const D8 &b)
{
    D8 r(a.v - b.v);
#pragma unroll
    for (int k = 0; k < kDir; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
VLCT_AD_FN D8 operator-(const D8 &a)
{
    D8 r(-a.v);
#pragma unroll
    for (int k = 0; k < kDir; ++k) r.d[k] = -a.d[k];
    return r;
}
VLCT_AD_FN D8 operator*(const D8 &a, const D8 &b)
{
    D8 r(a.v * b.v);
#pragma unroll
    for (int k = 0; k < kDir; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
VLCT_AD_FN D8 operator/(const D8 &a, const D8 &b)
{
    const double q = a.v / b.v;
    D8 r(q);
#pragma unroll
    for (int k = 0; k < kDir; ++k) r.d[k] = (a.d[k] - q * b.d[k]) / b.v;
    return r;
}
VLCT_AD_FN bool operator<(const D8 &a, const D8 &b) { return a.v < b.v; }
VLCT_AD_FN bool operator>(const D8 &a, const D8 &b) { return a.v > b.v; }
VLCT_AD_FN bool operator<=(const D8 &a, const D8 &b) { return a.v <= b.v; }
VLCT_AD_FN bool operator>=(const D8 &a, const D8 &b) { return a.v >= b.v; }
VLCT_AD_FN bool operator==(const D8 &a, const D8 &b) { return a.v == b.v; }
VLCT_AD_FN bool operator!=(const D8 &a, const D8 &b) { return a.v != b.v; }
VLCT_AD_FN D8 sqrt(const D8 &a)
{
    const double s = ::sqrt(a.v);
    D8 r(s);
    const double h = s > 0.0 ? 0.5 / s : 0.0;
#pragma unroll
    for (int k = 0; k < kDir; ++k) r.d[k] = a.d[k] * h;
    return r;
}
VLCT_AD_FN D8 fabs(const D8 &a)
{
    D8 r = a.v < 0.0 ? -a : a;
    r.v = ::fabs(a.v);
    return r;
}
VLCT_AD_FN D8 fmin(const D8 &a, const D8 &b) { return b.v < a.v ? b : a; }
VLCT_AD_FN D8 fmax(const D8 &a, const D8 &b) { return b.v > a.v ? b : a; }
// |a| with the sign of b (the sign of b is a branch, not differentiated)
VLCT_AD_FN D8 copysign(const D8 &a, const D8 &b)
{
    const bool flip = (::signbit(a.v) != 0) != (::signbit(b.v) != 0);
    return flip ? -a : a;
}
#undef VLCT_AD_FN

// the device physics of the step, instantiated on dual numbers
#define double D8
#include "mhd_physics.hpp"
#undef double

}  // namespace vlct_ad

namespace vlct {

using vlct_ad::D8;
using vlct_ad::kDir;
namespace phys = vlct_ad::vlct;

// cotangent arrays of one stage's transposes
struct AdStage {
    double *lf[3][7];     // face-flux cotangents, flux-array layout
    double *lw[8];        // primitive cotangents per interior cell (rho, v, P, B_cc)
    double *leref[3];     // -(v x B) cotangents per interior cell
    double *lrec[3][14];  // reconstruction cotangents per interior cell: fm (7), fp (7)
};

__device__ __forceinline__ int wrapc(int i, int n) { return map_cell(i, n, VLCT_BC_PERIODIC); }

__device__ __forceinline__ idx_t cell_of(const Geom &g, int i, int j, int k)
{
    return cell_store(g, wrapc(i, g.n[0]), wrapc(j, g.n[1]), wrapc(k, g.n[2]));
}

// lab component of the primitive array for sweep-frame slot s of axis d:
// (rho, v_n, v_t1, v_t2, P, B_t1, B_t2) -> (0, 1+d, 1+t1, 1+t2, 4, 5+t1, 5+t2)
__device__ __forceinline__ int lab_slot(int d, int s)
{
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    switch (s) {
    case 0: return 0;
    case 1: return 1 + d;
    case 2: return 1 + t1;
    case 3: return 1 + t2;
    case 4: return 4;
    case 5: return 5 + t1;
    default: return 5 + t2;
    }
}
// lab conserved cell variable of sweep-frame flux component c of axis d
__device__ __forceinline__ int lab_cons(int d, int c)
{
    if (c == 0 || c == 4) return c;
    return 1 + (c == 1 ? d : (c == 2 ? (d + 1) % 3 : (d + 2) % 3));
}

__device__ __forceinline__ phys::W7 w7_dual(const Prims &P, int d, idx_t o)
{
    phys::W7 w;
    D8 *x[7] = {&w.d, &w.u, &w.v, &w.w, &w.p, &w.by, &w.bz};
#pragma unroll
    for (int s = 0; s < 7; ++s) *x[s] = D8(P.w[lab_slot(d, s)][o]);
    return w;
}

__global__ void k_ad_fill(double *p, idx_t n, double v)
{
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// lam_next = lam_out with each periodic duplicate face folded into face 0 (the
// step writes face n as a copy of face 0); lam_in starts as lam_next (U^{n+1}
// contains U^n with unit weight)
__global__ void k_ad_init(Geom g, StateP lo, StateW next, StateW lin)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N)
        for (int f = 0; f < 5; ++f) {
            next.u[f][t] = lo.u[f][t];
            lin.u[f][t] = lo.u[f][t];
        }
    for (int d = 0; d < 3; ++d) {
        const idx_t nf = N / g.n[d] * (g.n[d] + 1);
        if (t >= nf) continue;
        const int nx = g.n[0] + (d == 0), ny = g.n[1] + (d == 1);
        const int i = (int)(t % nx), j = (int)((t / nx) % ny), k = (int)(t / ((idx_t)nx * ny));
        const int e[3] = {i, j, k};
        double v = lo.b[d][t];
        if (e[d] == g.n[d]) v = 0.0;  // the duplicate itself carries nothing
        if (e[d] == 0) {
            int q[3] = {i, j, k};
            q[d] = g.n[d];
            v += lo.b[d][face_store(g, d, q[0], q[1], q[2])];
        }
        next.b[d][t] = v;
        lin.b[d][t] = v;
    }
}

// acc += add (cells and faces)
__global__ void k_ad_add(Geom g, StateW acc, StateP add)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N)
        for (int f = 0; f < 5; ++f) acc.u[f][t] += add.u[f][t];
    for (int d = 0; d < 3; ++d) {
        const idx_t nf = N / g.n[d] * (g.n[d] + 1);
        if (t < nf) acc.b[d][t] += add.b[d][t];
    }
}

// hydro flux cotangents of the faces of axis D from the cell cotangents of the
// stage output: u_i -= c (F(i+1/2) - F(i-1/2)) with c = factor dt / d_D
template <int D>
__global__ void k_ad_flux_hydro(Geom g, StateP lout, AdStage A, const double *dt_dev,
                                double factor)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const int i = (int)(t % g.n[0]), j = (int)((t / g.n[0]) % g.n[1]),
              k = (int)(t / ((idx_t)g.n[0] * g.n[1]));
    int lw[3] = {i, j, k};
    lw[D] -= 1;
    const idx_t cr = t, cl = cell_of(g, lw[0], lw[1], lw[2]);
    const double c = factor * dt_dev[0] / g.dl[D];
    const idx_t o = fidx(g, D, i, j, k);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int f = lab_cons(D, q);
        A.lf[D][q][o] = c * (lout.u[f][cr] - lout.u[f][cl]);
    }
}

__device__ __forceinline__ void upwind_weights(double s, double &lo, double &hi)
{
    lo = s > 0.0 ? 1.0 : (s < 0.0 ? 0.0 : 0.5);
    hi = 1.0 - lo;
}

// edge fields of component A from the face cotangents of the stage output
// (curl transposed), then the edge-field formula transposed with the upwind
// weights of the forward fluxes: face-EMF and reference-field cotangents
template <int A>
__global__ void k_ad_edges(Geom g, StateP lout, Flux F, AdStage S, const double *dt_dev,
                           double factor)
{
    constexpr int B = (A + 1) % 3, C = (A + 2) % 3;
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const int i = (int)(t % g.n[0]), j = (int)((t / g.n[0]) % g.n[1]),
              k = (int)(t / ((idx_t)g.n[0] * g.n[1]));
    const double cx = factor * dt_dev[0] / g.dl[0], cy = factor * dt_dev[0] / g.dl[1],
                 cz = factor * dt_dev[0] / g.dl[2];
    auto lb = [&](int d, int a, int b2, int c2) {
        return lout.b[d][face_store(g, d, wrapc(a, g.n[0]), wrapc(b2, g.n[1]), wrapc(c2, g.n[2]))];
    };
    double le;
    if (A == 2)
        le = cy * (lb(0, i, j, k) - lb(0, i, j - 1, k)) + cx * (lb(1, i - 1, j, k) - lb(1, i, j, k));
    else if (A == 0)
        le = cz * (lb(1, i, j, k) - lb(1, i, j, k - 1)) + cy * (lb(2, i, j - 1, k) - lb(2, i, j, k));
    else
        le = cz * (lb(0, i, j, k - 1) - lb(0, i, j, k)) + cx * (lb(2, i, j, k) - lb(2, i - 1, j, k));
    if (le == 0.0) return;
    int x0[3] = {i, j, k}, xb[3] = {i, j, k}, xc[3] = {i, j, k}, xbc[3] = {i, j, k};
    xb[B] -= 1;
    xc[C] -= 1;
    xbc[B] -= 1;
    xbc[C] -= 1;
    const idx_t fb_c = fidx(g, B, x0[0], x0[1], x0[2]), fb_cm = fidx(g, B, xc[0], xc[1], xc[2]);
    const idx_t fc_b = fidx(g, C, x0[0], x0[1], x0[2]), fc_bm = fidx(g, C, xb[0], xb[1], xb[2]);
    double w1l, w1h, w2l, w2h, w3l, w3h, w4l, w4h;
    upwind_weights(F.f[B][7][fb_c], w1l, w1h);
    upwind_weights(F.f[B][7][fb_cm], w2l, w2h);
    upwind_weights(F.f[C][7][fc_b], w3l, w3h);
    upwind_weights(F.f[C][7][fc_bm], w4l, w4h);
    // eb = -F_B[B_t1], ec = +F_C[B_t2]
    atomicAdd(&S.lf[B][5][fb_c], -0.25 * (1.0 + w3h + w4h) * le);
    atomicAdd(&S.lf[B][5][fb_cm], -0.25 * (1.0 + w3l + w4l) * le);
    atomicAdd(&S.lf[C][6][fc_b], 0.25 * (1.0 + w1h + w2h) * le);
    atomicAdd(&S.lf[C][6][fc_bm], 0.25 * (1.0 + w1l + w2l) * le);
    atomicAdd(&S.leref[A][cell_of(g, x0[0], x0[1], x0[2])], -0.25 * (w1h + w3h) * le);
    atomicAdd(&S.leref[A][cell_of(g, xb[0], xb[1], xb[2])], -0.25 * (w1l + w4h) * le);
    atomicAdd(&S.leref[A][cell_of(g, xc[0], xc[1], xc[2])], -0.25 * (w2h + w3l) * le);
    atomicAdd(&S.leref[A][cell_of(g, xbc[0], xbc[1], xbc[2])], -0.25 * (w2l + w4l) * le);
}

// periodic copies of a face (the normal index n and the transverse ghost rows
// -1 and n of the flux arrays) add their cotangent to the face itself
template <int D>
__global__ void k_ad_fold(Geom g, AdStage S)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const int e[3] = {(int)(t % g.n[0]), (int)((t / g.n[0]) % g.n[1]),
                      (int)(t / ((idx_t)g.n[0] * g.n[1]))};
    const idx_t self = fidx(g, D, e[0], e[1], e[2]);
    for (int c = 5; c < 7; ++c) {
        double acc = 0.0;
        for (int m0 = -1; m0 <= 1; ++m0)
            for (int m1 = -1; m1 <= 1; ++m1)
                for (int m2 = -1; m2 <= 1; ++m2) {
                    const int m[3] = {m0, m1, m2};
                    int q[3];
                    bool ok = !(m0 == 0 && m1 == 0 && m2 == 0);
                    for (int a = 0; a < 3; ++a) {
                        q[a] = e[a] + m[a] * g.n[a];
                        const int lo = a == D ? 0 : -1, hi = g.n[a];
                        if (q[a] < lo || q[a] > hi) ok = false;
                    }
                    if (ok) acc += S.lf[D][c][fidx(g, D, q[0], q[1], q[2])];
                }
        S.lf[D][c][self] += acc;
    }
}

// -(v x B) at cell centres transposed into the primitive cotangents
__global__ void k_ad_eref(Geom g, Prims P, AdStage S)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const int i = (int)(t % g.n[0]), j = (int)((t / g.n[0]) % g.n[1]),
              k = (int)(t / ((idx_t)g.n[0] * g.n[1]));
    const idx_t o = pidx(g, i, j, k);
    const double vx = P.w[1][o], vy = P.w[2][o], vz = P.w[3][o];
    const double bx = P.w[5][o], by = P.w[6][o], bz = P.w[7][o];
    const double ex = S.leref[0][t], ey = S.leref[1][t], ez = S.leref[2][t];
    S.lw[1][t] += bz * ey - by * ez;
    S.lw[2][t] += -bz * ex + bx * ez;
    S.lw[3][t] += by * ex - bx * ey;
    S.lw[5][t] += -vz * ey + vy * ez;
    S.lw[6][t] += vz * ex - vx * ez;
    S.lw[7][t] += -vy * ex + vx * ey;
}

// interface states of the face between cells (i-1) and i along D (the
// reconstruction of each cell, on dual numbers with zero derivatives)
template <int D, int RECON>
__device__ __forceinline__ void face_states(const Geom &g, const Prims &P, int i, int j, int k,
                                            phys::W7 &wl, phys::W7 &wr)
{
    auto at = [&](int off) {
        int q[3] = {i, j, k};
        q[D] += off;
        return pidx(g, q[0], q[1], q[2]);
    };
    if (RECON == VLCT_RECON_PCM) {
        wl = w7_dual(P, D, at(-1));
        wr = w7_dual(P, D, at(0));
        return;
    }
    constexpr bool kChar = RECON == VLCT_RECON_PLMC;
    phys::W7 fm, fp;
    phys::plmc<kChar>(w7_dual(P, D, at(-2)), w7_dual(P, D, at(-1)), w7_dual(P, D, at(0)),
                      D8(P.w[5 + D][at(-1)]), D8(g.gamma), fm, wl);
    phys::floor_state(wl);
    phys::plmc<kChar>(w7_dual(P, D, at(-1)), w7_dual(P, D, at(0)), w7_dual(P, D, at(1)),
                      D8(P.w[5 + D][at(0)]), D8(g.gamma), wr, fp);
    phys::floor_state(wr);
}

// HLLD of the faces of axis D transposed: (lam W_L, lam W_R, lam B_n) =
// J^T lam F, the Jacobian formed by dual numbers over the 15 inputs.  PCM: the
// states are cell primitives (atomics into the primitive cotangents);
// otherwise they are reconstruction outputs (each written once).
template <int D, int RECON>
__global__ __launch_bounds__(kBlock) void k_ad_hlld(Geom g, Prims P, StateP st, AdStage S, StateW lacc)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const int i = (int)(t % g.n[0]), j = (int)((t / g.n[0]) % g.n[1]),
              k = (int)(t / ((idx_t)g.n[0] * g.n[1]));
    int e[3] = {i, j, k};
    const idx_t o = fidx(g, D, i, j, k);
    double lfl[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) lfl[c] = S.lf[D][c][o];
    const idx_t fo = face_store(g, D, i, j, k);
    const double bn = st.b[D][fo];
    phys::W7 wl0, wr0;
    face_states<D, RECON>(g, P, e[0], e[1], e[2], wl0, wr0);
    double x[15];
    {
        const D8 *a[7] = {&wl0.d, &wl0.u, &wl0.v, &wl0.w, &wl0.p, &wl0.by, &wl0.bz};
        const D8 *b[7] = {&wr0.d, &wr0.u, &wr0.v, &wr0.w, &wr0.p, &wr0.by, &wr0.bz};
        for (int s = 0; s < 7; ++s) {
            x[s] = a[s]->v;
            x[7 + s] = b[s]->v;
        }
        x[14] = bn;
    }
    double grad[16];
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        D8 in[15];
#pragma unroll
        for (int q = 0; q < 15; ++q) {
            in[q] = D8(x[q]);
            const int kk = q - pass * kDir;
            if (kk >= 0 && kk < kDir) in[q].d[kk] = 1.0;
        }
        const phys::W7 wl{in[0], in[1], in[2], in[3], in[4], in[5], in[6]};
        const phys::W7 wr{in[7], in[8], in[9], in[10], in[11], in[12], in[13]};
        D8 f[7], upw;
        phys::hlld(wl, wr, in[14], D8(g.gamma), D8(g.gm1i), f, upw);
#pragma unroll
        for (int kk = 0; kk < kDir; ++kk) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < 7; ++c) s += lfl[c] * f[c].d[kk];
            if (pass * kDir + kk < 16) grad[pass * kDir + kk] = s;
        }
    }
    // the face's stored normal field
    lacc.b[D][fo] += grad[14];
    if (RECON == VLCT_RECON_PCM) {
        int l[3] = {i, j, k};
        l[D] -= 1;
        const idx_t cl = cell_of(g, l[0], l[1], l[2]);
        for (int s = 0; s < 7; ++s) {
            atomicAdd(&S.lw[lab_slot(D, s)][cl], grad[s]);
            atomicAdd(&S.lw[lab_slot(D, s)][t], grad[7 + s]);
        }
    } else {
        int l[3] = {i, j, k};
        l[D] -= 1;
        const idx_t cl = cell_of(g, l[0], l[1], l[2]);
        for (int s = 0; s < 7; ++s) {
            S.lrec[D][7 + s][cl] = grad[s];  // high face (fp) of the left cell
            S.lrec[D][s][t] = grad[7 + s];   // low face (fm) of the right cell
        }
    }
}

// reconstruction of each cell along D transposed over its 22 inputs (three
// stencil states and the cell's B_cc,D); the floors of the interface states
// are part of it
template <int D, int RECON>
__global__ __launch_bounds__(kBlock) void k_ad_recon(Geom g, Prims P, AdStage S)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const int i = (int)(t % g.n[0]), j = (int)((t / g.n[0]) % g.n[1]),
              k = (int)(t / ((idx_t)g.n[0] * g.n[1]));
    constexpr bool kChar = RECON == VLCT_RECON_PLMC;
    double lr[14];
    for (int c = 0; c < 14; ++c) lr[c] = S.lrec[D][c][t];
    idx_t po[3];
    for (int q = 0; q < 3; ++q) {
        int e[3] = {i, j, k};
        e[D] += q - 1;
        po[q] = pidx(g, e[0], e[1], e[2]);
    }
    double x[22];
    for (int q = 0; q < 3; ++q)
        for (int s = 0; s < 7; ++s) x[7 * q + s] = P.w[lab_slot(D, s)][po[q]];
    x[21] = P.w[5 + D][po[1]];
    double grad[24];
#pragma unroll
    for (int pass = 0; pass < 3; ++pass) {
        D8 in[22];
#pragma unroll
        for (int q = 0; q < 22; ++q) {
            in[q] = D8(x[q]);
            const int kk = q - pass * kDir;
            if (kk >= 0 && kk < kDir) in[q].d[kk] = 1.0;
        }
        const phys::W7 wm{in[0], in[1], in[2], in[3], in[4], in[5], in[6]};
        const phys::W7 w0{in[7], in[8], in[9], in[10], in[11], in[12], in[13]};
        const phys::W7 wp{in[14], in[15], in[16], in[17], in[18], in[19], in[20]};
        phys::W7 fm, fp;
        phys::plmc<kChar>(wm, w0, wp, in[21], D8(g.gamma), fm, fp);
        phys::floor_state(fm);
        phys::floor_state(fp);
        const D8 *o[14] = {&fm.d, &fm.u, &fm.v, &fm.w, &fm.p, &fm.by, &fm.bz,
                           &fp.d, &fp.u, &fp.v, &fp.w, &fp.p, &fp.by, &fp.bz};
#pragma unroll
        for (int kk = 0; kk < kDir; ++kk) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < 14; ++c) s += lr[c] * o[c]->d[kk];
            if (pass * kDir + kk < 24) grad[pass * kDir + kk] = s;
        }
    }
    for (int q = 0; q < 3; ++q) {
        int e[3] = {i, j, k};
        e[D] += q - 1;
        const idx_t c = cell_of(g, e[0], e[1], e[2]);
        for (int s = 0; s < 7; ++s) atomicAdd(&S.lw[lab_slot(D, s)][c], grad[7 * q + s]);
    }
    atomicAdd(&S.lw[5 + D][t], grad[21]);
}

// primitive recovery (Sec. 2.1; B_cc = face average) transposed into the
// cotangents of the stage's conserved cells and faces; a floored quantity is
// a constant
__global__ void k_ad_prims(Geom g, StateP st, AdStage S, StateW lacc)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const int i = (int)(t % g.n[0]), j = (int)((t / g.n[0]) % g.n[1]),
              k = (int)(t / ((idx_t)g.n[0] * g.n[1]));
    const idx_t fl[3] = {face_store(g, 0, i, j, k), face_store(g, 1, i, j, k),
                         face_store(g, 2, i, j, k)};
    const idx_t fh[3] = {face_store(g, 0, wrapc(i + 1, g.n[0]), j, k),
                         face_store(g, 1, i, wrapc(j + 1, g.n[1]), k),
                         face_store(g, 2, i, j, wrapc(k + 1, g.n[2]))};
    double bc[3];
    for (int d = 0; d < 3; ++d) bc[d] = 0.5 * (st.b[d][fl[d]] + st.b[d][fh[d]]);
    double d = st.u[0][t];
    const bool dfloor = !(d >= 1.0e-20);
    if (dfloor) d = 1.0e-20;
    const double id = 1.0 / d;
    const double v[3] = {st.u[1][t] * id, st.u[2][t] * id, st.u[3][t] * id};
    const double ke = 0.5 * d * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double me = 0.5 * (bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
    const double p = (g.gamma - 1.0) * (st.u[4][t] - ke - me);
    const bool pfloor = !(p >= 1.0e-20);
    const double gm1 = g.gamma - 1.0;
    const double lr = S.lw[0][t], lp = pfloor ? 0.0 : S.lw[4][t];
    const double lv[3] = {S.lw[1][t], S.lw[2][t], S.lw[3][t]};
    const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double lrho = dfloor ? 0.0 : lr + lp * gm1 * 0.5 * v2;
    for (int l = 0; l < 3; ++l) {
        if (!dfloor) lrho -= lv[l] * v[l] * id;
        lacc.u[1 + l][t] += lv[l] * id - lp * gm1 * v[l];
    }
    lacc.u[0][t] += lrho;
    lacc.u[4][t] += lp * gm1;
    for (int l = 0; l < 3; ++l) {
        const double lb = 0.5 * (S.lw[5 + l][t] - lp * gm1 * bc[l]);
        atomicAdd(&lacc.b[l][fl[l]], lb);
        atomicAdd(&lacc.b[l][fh[l]], lb);
    }
}

static unsigned cells_grid(const Geom &g)
{
    return nblocks((size_t)g.n[0] * g.n[1] * g.n[2]);
}

static void fill(double *p, size_t n, hipStream_t s)
{
    if (n) k_ad_fill<<<nblocks(n), kBlock, 0, s>>>(p, (idx_t)n, 0.0);
}

// transposes of one stage: lout is the cotangent of the stage's output state,
// st/P/F the stage's input state, primitives and forward fluxes; the result
// is added to lacc (the cotangent of the stage's input state)
static void stage_adjoint(const Geom &g, double factor, const StateP &lout, const StateP &st,
                          const Prims &P, const Flux &F, int recon, const AdStage &S,
                          const StateW &lacc, size_t flux_len[3], const double *dt,
                          hipStream_t s)
{
    const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 7; ++c) fill(S.lf[d][c], flux_len[d], s);
    for (int f = 0; f < 8; ++f) fill(S.lw[f], N, s);
    for (int a = 0; a < 3; ++a) fill(S.leref[a], N, s);
    const unsigned gc = cells_grid(g);
    k_ad_flux_hydro<0><<<gc, kBlock, 0, s>>>(g, lout, S, dt, factor);
    k_ad_flux_hydro<1><<<gc, kBlock, 0, s>>>(g, lout, S, dt, factor);
    k_ad_flux_hydro<2><<<gc, kBlock, 0, s>>>(g, lout, S, dt, factor);
    k_ad_edges<0><<<gc, kBlock, 0, s>>>(g, lout, F, S, dt, factor);
    k_ad_edges<1><<<gc, kBlock, 0, s>>>(g, lout, F, S, dt, factor);
    k_ad_edges<2><<<gc, kBlock, 0, s>>>(g, lout, F, S, dt, factor);
    k_ad_fold<0><<<gc, kBlock, 0, s>>>(g, S);
    k_ad_fold<1><<<gc, kBlock, 0, s>>>(g, S);
    k_ad_fold<2><<<gc, kBlock, 0, s>>>(g, S);
    k_ad_eref<<<gc, kBlock, 0, s>>>(g, P, S);
#define VLCT_AD_HLLD(R)                                                        \
    k_ad_hlld<0, R><<<gc, kBlock, 0, s>>>(g, P, st, S, lacc);                  \
    k_ad_hlld<1, R><<<gc, kBlock, 0, s>>>(g, P, st, S, lacc);                  \
    k_ad_hlld<2, R><<<gc, kBlock, 0, s>>>(g, P, st, S, lacc);
#define VLCT_AD_RECON(R)                                                       \
    k_ad_recon<0, R><<<gc, kBlock, 0, s>>>(g, P, S);                           \
    k_ad_recon<1, R><<<gc, kBlock, 0, s>>>(g, P, S);                           \
    k_ad_recon<2, R><<<gc, kBlock, 0, s>>>(g, P, S);
    if (recon == VLCT_RECON_PCM) {
        VLCT_AD_HLLD(VLCT_RECON_PCM)
    } else if (recon == VLCT_RECON_PLMC) {
        VLCT_AD_HLLD(VLCT_RECON_PLMC)
        VLCT_AD_RECON(VLCT_RECON_PLMC)
    } else {
        VLCT_AD_HLLD(VLCT_RECON_PLMP)
        VLCT_AD_RECON(VLCT_RECON_PLMP)
    }
#undef VLCT_AD_HLLD
#undef VLCT_AD_RECON
    k_ad_prims<<<gc, kBlock, 0, s>>>(g, st, S, lacc);
}

// workspace of the adjoint: forward intermediates and cotangents
struct AdLayout {
    size_t prims[2], half[8], flux[2][3], lnext[8], lhalf[8], lf[3], lw, leref, lrec[3], total;
    size_t prims_len, flux_len[3];
};

static size_t ad_align(size_t x) { return (x + 255) & ~(size_t)255; }

static AdLayout ad_layout(const Geom &g)
{
    AdLayout L;
    size_t off = 0;
    const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    L.prims_len = (size_t)g.p[0] * g.p[1] * g.p[2];
    for (int h = 0; h < 2; ++h) {
        L.prims[h] = off;
        off += 8 * ad_align(L.prims_len * 8);
    }
    for (int f = 0; f < 8; ++f) {
        L.half[f] = off;
        off += ad_align(field_len(g.n, f) * 8);
    }
    for (int d = 0; d < 3; ++d)
        L.flux_len[d] = (size_t)flux_dim(g.n, d, 0) * flux_dim(g.n, d, 1) * flux_dim(g.n, d, 2);
    for (int h = 0; h < 2; ++h)
        for (int d = 0; d < 3; ++d) {
            L.flux[h][d] = off;
            off += 8 * ad_align(L.flux_len[d] * 8);
        }
    for (int f = 0; f < 8; ++f) {
        L.lnext[f] = off;
        off += ad_align(field_len(g.n, f) * 8);
    }
    for (int f = 0; f < 8; ++f) {
        L.lhalf[f] = off;
        off += ad_align(field_len(g.n, f) * 8);
    }
    for (int d = 0; d < 3; ++d) {
        L.lf[d] = off;
        off += 7 * ad_align(L.flux_len[d] * 8);
    }
    L.lw = off;
    off += 8 * ad_align(N * 8);
    L.leref = off;
    off += 3 * ad_align(N * 8);
    for (int d = 0; d < 3; ++d) {
        L.lrec[d] = off;
        off += 14 * ad_align(N * 8);
    }
    L.total = off;
    return L;
}

}  // namespace vlct

using namespace vlct;

extern "C" {

size_t vlct_adjoint_workspace_bytes(const vlct_grid *g)
{
    if (!grid_ok(g)) return 0;
    return ad_layout(make_geom(g)).total;
}

int vlct_step_adjoint(const vlct_grid *vg, const vlct_state *in, const vlct_state *lam_out,
                      const vlct_state *lam_in, const double *dt_dev, void *ws, size_t ws_bytes,
                      void *stream)
{
    if (!grid_ok(vg) || !state_ok(in) || !state_ok(lam_out) || !state_ok(lam_in) || !dt_dev)
        return VLCT_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (vg->bc[d] != VLCT_BC_PERIODIC) return VLCT_EUNSUPPORTED;
    if (vg->recon != VLCT_RECON_PCM && vg->recon != VLCT_RECON_PLMC && vg->recon != VLCT_RECON_PLMP)
        return VLCT_EUNSUPPORTED;
    {
        // no array of lam_in may overlap an array of `in` or `lam_out`, nor another of lam_in
        const int n[3] = {vg->nx, vg->ny, vg->nz};
        const vlct_state *sts[3] = {lam_in, in, lam_out};
        uintptr_t lo[3][8], hi[3][8];
        for (int q = 0; q < 3; ++q) {
            const double *p[8] = {sts[q]->rho, sts[q]->mx, sts[q]->my, sts[q]->mz, sts[q]->E,
                                  sts[q]->bx, sts[q]->by, sts[q]->bz};
            for (int f = 0; f < 8; ++f) {
                lo[q][f] = reinterpret_cast<uintptr_t>(p[f]);
                hi[q][f] = lo[q][f] + field_len(n, f) * sizeof(double);
            }
        }
        for (int f = 0; f < 8; ++f)
            for (int q = 0; q < 3; ++q)
                for (int h = 0; h < 8; ++h) {
                    if (q == 0 && h == f) continue;
                    if (lo[0][f] < hi[q][h] && lo[q][h] < hi[0][f]) return VLCT_EINVAL;
                }
    }
    const Geom g = make_geom(vg);
    AdLayout L = ad_layout(g);
    if (!ws || ws_bytes < L.total) return VLCT_EWORKSPACE;
    char *b = static_cast<char *>(ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto arr = [&](size_t off) { return reinterpret_cast<double *>(b + off); };
    Prims P[2];
    for (int h = 0; h < 2; ++h)
        for (int f = 0; f < 8; ++f) P[h].w[f] = arr(L.prims[h] + f * ad_align(L.prims_len * 8));
    StateW half, lnext, lhalf;
    for (int f = 0; f < 8; ++f) {
        double *a = arr(L.half[f]), *c = arr(L.lnext[f]), *e = arr(L.lhalf[f]);
        if (f < 5) { half.u[f] = a; lnext.u[f] = c; lhalf.u[f] = e; }
        else { half.b[f - 5] = a; lnext.b[f - 5] = c; lhalf.b[f - 5] = e; }
    }
    Flux F[2];
    for (int h = 0; h < 2; ++h)
        for (int d = 0; d < 3; ++d)
            for (int c = 0; c < 8; ++c)
                F[h].f[d][c] = arr(L.flux[h][d] + c * ad_align(L.flux_len[d] * 8));
    AdStage S;
    const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 7; ++c) S.lf[d][c] = arr(L.lf[d] + c * ad_align(L.flux_len[d] * 8));
    for (int f = 0; f < 8; ++f) S.lw[f] = arr(L.lw + f * ad_align(N * 8));
    for (int a = 0; a < 3; ++a) S.leref[a] = arr(L.leref + a * ad_align(N * 8));
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 14; ++c) S.lrec[d][c] = arr(L.lrec[d] + c * ad_align(N * 8));

    // forward intermediates at U^n (same kernels as vlct_step)
    const StateP sin = as_const(in);
    int rc = launch_prims(g, sin, P[0], nullptr, s);
    if (!rc) rc = launch_fluxes(g, sin, P[0], F[0], VLCT_RECON_PCM, nullptr, s);
    if (!rc) rc = launch_ct(g, false, P[0], F[0], sin, half, dt_dev, nullptr, s);
    const StateP hc = as_const(half);
    if (!rc) rc = launch_prims(g, hc, P[1], nullptr, s);
    if (!rc) rc = launch_fluxes(g, hc, P[1], F[1], vg->recon, nullptr, s);
    if (rc) return rc;

    // reverse: U^{n+1} = U^n + (corrector increment); U^{n+1/2} = U^n + (predictor increment)
    const StateW lin = as_mut(lam_in);
    const unsigned gf = nblocks((size_t)(g.n[0] + 1) * (g.n[1] + 1) * (g.n[2] + 1));
    k_ad_init<<<gf, kBlock, 0, s>>>(g, as_const(lam_out), lnext, lin);
    for (int f = 0; f < 5; ++f) fill(lhalf.u[f], N, s);
    for (int d = 0; d < 3; ++d) fill(lhalf.b[d], field_len(g.n, 5 + d), s);
    stage_adjoint(g, 1.0, as_const(lnext), hc, P[1], F[1], vg->recon, S, lhalf, L.flux_len,
                  dt_dev, s);
    k_ad_add<<<gf, kBlock, 0, s>>>(g, lin, as_const(lhalf));
    stage_adjoint(g, 0.5, as_const(lhalf), sin, P[0], F[0], VLCT_RECON_PCM, S, lin, L.flux_len,
                  dt_dev, s);
    return hipGetLastError() == hipSuccess ? VLCT_OK : VLCT_EHIP;
}

}  // extern "C"
