// vlct_adjoint.hip -- adjoint (reverse derivative) of one VL+CT step (Caddy &
// Schneider, "Cholla-MHD", Sec. 2.2) on gfx950:
//
//   lam_in = (d U^{n+1} / d U^n)^T lam_out
//
// for a step of fixed size dt (dt is a parameter, not differentiated), with
// every branch (HLLD wave regions, limiter cases, CT upwind sides, floors)
// taken as in the forward evaluation at U^n.  The step is the composition
//   U^n -> W^n -> PCM/HLLD fluxes -> CT edge fields -> U^{n+1/2}
//       -> W^{n+1/2} -> reconstruction/HLLD fluxes -> CT edge fields -> U^{n+1}
// with U^{n+1/2} = U^n + G1(U^n) and U^{n+1} = U^n + G2(U^{n+1/2}), so
//   lam_in = lam + mu + G1'^T mu,   mu = G2'^T lam.
// Each stage transpose runs, per cell or face and without a tape:
//   edges   : edge-field cotangents from the face cotangents (curl transposed)
//   faces   : flux cotangents (flux differences transposed; B_t1/B_t2 fluxes
//             gathered from the two edges that use each, with the upwind
//             weights of the forward fluxes), then HLLD reversed (the y and
//             z faces of a reconstructing stage by column marches that
//             reconstruct each cell once)
//   recon   : PLMC/PLMP/PPMC/PPMP reversed per cell and axis (corrector only)
//   prims   : reference fields -(v x B) gathered from the 12 edges around the
//             cell and reversed, then primitive recovery reversed
// The forward intermediates (primitives, fluxes with their upwind indicators,
// the half-step state) are recomputed by the step's own kernels.  Periodic
// boundaries: a ghost cell or ghost flux row holds exactly the values of its
// periodic image, so every cotangent is accumulated on the image directly.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "vlct_common.hpp"
#include "mhd_adjoint.hpp"

namespace vlct {

// cotangent arrays of one stage's transposes (interior cells, cell_store order)
struct AdStage {
    double *le[3];        // edge fields E_A at the edge indexed like its cell
    uint32_t *wcode;      // upwind sides of the edges' four faces, 8 bits per component
    double *lw[8];        // primitives (rho, v, P, B_cc)
    double *lrec[3][14];  // interface states per axis: low face (7), high face (7)
};

__device__ __forceinline__ int wrapc(int i, int n) { return map_cell(i, n, VLCT_BC_PERIODIC); }

__device__ __forceinline__ idx_t cell_of(const Geom &g, int i, int j, int k)
{
    return cell_store(g, wrapc(i, g.n[0]), wrapc(j, g.n[1]), wrapc(k, g.n[2]));
}
__device__ __forceinline__ idx_t cell_of(const Geom &g, const int x[3])
{
    return cell_of(g, x[0], x[1], x[2]);
}
__device__ __forceinline__ void cell_coords(const Geom &g, idx_t t, int x[3])
{
    x[0] = (int)(t % g.n[0]);
    x[1] = (int)((t / g.n[0]) % g.n[1]);
    x[2] = (int)(t / ((idx_t)g.n[0] * g.n[1]));
}

// lab component of the primitive array for sweep-frame slot s of axis d:
// (rho, v_n, v_t1, v_t2, P, B_t1, B_t2) -> (0, 1+d, 1+t1, 1+t2, 4, 5+t1, 5+t2)
__host__ __device__ __forceinline__ int lab_slot(int d, int s)
{
    if (s == 0 || s == 4) return s;
    const int off = s < 4 ? 1 : 5;
    const int r = s < 4 ? s - 1 : s - 5 + 1;  // 0 normal, 1 t1, 2 t2
    return off + (d + r) % 3;
}
// lab conserved cell variable of sweep-frame flux component c (< 5) of axis d
__host__ __device__ __forceinline__ int lab_cons(int d, int c)
{
    if (c == 0 || c == 4) return c;
    return 1 + (d + c - 1) % 3;
}

__device__ __forceinline__ W7 w7_at(const Prims &P, int d, idx_t o)
{
    return W7{P.w[0][o], P.w[lab_slot(d, 1)][o], P.w[lab_slot(d, 2)][o], P.w[lab_slot(d, 3)][o],
              P.w[4][o], P.w[lab_slot(d, 5)][o], P.w[lab_slot(d, 6)][o]};
}

// upwind sides of one stage's interior faces (side_code, per axis, at the
// index of the cell whose low face it is)
struct Sides {
    const uint8_t *s[3];
};

// 8-bit code of edge (A, x0): the sides of the faces F_B(x0), F_B(x0 - e_C),
// F_C(x0), F_C(x0 - e_B) (the four upwind terms of the edge field)
template <int A>
__device__ __forceinline__ uint32_t edge_code(const Geom &g, const Sides &sd, const int x0[3])
{
    constexpr int B = (A + 1) % 3, C = (A + 2) % 3;
    int xb[3] = {x0[0], x0[1], x0[2]}, xc[3] = {x0[0], x0[1], x0[2]};
    xb[B] -= 1;
    xc[C] -= 1;
    return (uint32_t)sd.s[B][cell_of(g, x0)] | ((uint32_t)sd.s[B][cell_of(g, xc)] << 2) |
           ((uint32_t)sd.s[C][cell_of(g, x0)] << 4) | ((uint32_t)sd.s[C][cell_of(g, xb)] << 6);
}

// upwind weights of edge (A, x0): w[0..7] = w1l, w1h, w2l, w2h, w3l, w3h, w4l, w4h
template <int A>
__device__ __forceinline__ void edge_weights(const Geom &g, const AdStage &S, const int x0[3],
                                             double w[8])
{
    const uint32_t c = S.wcode[cell_of(g, x0)] >> (8 * A);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t k = (c >> (2 * q)) & 3u;
        w[2 * q] = k == 0u ? 1.0 : (k == 1u ? 0.0 : 0.5);
        w[2 * q + 1] = 1.0 - w[2 * q];
    }
}

// lam_next = lam_out with each periodic duplicate face folded into face 0 (the
// step writes face n as a copy of face 0); the half-step cotangent `half`
// starts at zero
__global__ void k_ad_init(Geom g, StateP lo, StateW next, StateW half)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N)
        for (int f = 0; f < 5; ++f) {
            next.u[f][t] = lo.u[f][t];
            half.u[f][t] = 0.0;
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
        half.b[d][t] = 0.0;
    }
}

// out = a + b (cells and faces): lam_in starts as lam_next (U^{n+1} contains
// U^n with unit weight) plus the half-step cotangent
__global__ void k_ad_add(Geom g, StateW out, StateP a, StateP b)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N)
        for (int f = 0; f < 5; ++f) out.u[f][t] = a.u[f][t] + b.u[f][t];
    for (int d = 0; d < 3; ++d) {
        const idx_t nf = N / g.n[d] * (g.n[d] + 1);
        if (t < nf) out.b[d][t] = a.b[d][t] + b.b[d][t];
    }
}

// edge-field cotangents (curl of the face update transposed): the face update
// is b_x -= cy (Ez(j+1) - Ez(j)) - cz (Ey(k+1) - Ey(k)) and cyclically
// zero_lw: also clears the cell's primitive cotangents S.lw, into which the
// reconstruction transposes that follow add
__global__ void k_ad_edges(Geom g, StateP lout, Sides sd, AdStage S, const double *dt_dev,
                           double factor, int zero_lw)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    int x[3];
    cell_coords(g, t, x);
    const int i = x[0], j = x[1], k = x[2];
    const double cx = factor * dt_dev[0] / g.dl[0], cy = factor * dt_dev[0] / g.dl[1],
                 cz = factor * dt_dev[0] / g.dl[2];
    auto lb = [&](int d, int a, int b2, int c2) {
        return lout.b[d][face_store(g, d, wrapc(a, g.n[0]), wrapc(b2, g.n[1]), wrapc(c2, g.n[2]))];
    };
    S.le[0][t] = cz * (lb(1, i, j, k) - lb(1, i, j, k - 1)) + cy * (lb(2, i, j - 1, k) - lb(2, i, j, k));
    S.le[1][t] = cz * (lb(0, i, j, k - 1) - lb(0, i, j, k)) + cx * (lb(2, i, j, k) - lb(2, i - 1, j, k));
    S.le[2][t] = cy * (lb(0, i, j, k) - lb(0, i, j - 1, k)) + cx * (lb(1, i - 1, j, k) - lb(1, i, j, k));
    S.wcode[t] = edge_code<0>(g, sd, x) | (edge_code<1>(g, sd, x) << 8) | (edge_code<2>(g, sd, x) << 16);
    if (zero_lw)
        for (int f = 0; f < 8; ++f) S.lw[f][t] = 0.0;
}

// cotangents of the 7 fluxes of the face of axis D at x (the low face of cell x)
template <int D>
__device__ __forceinline__ void flux_cotangent(const Geom &g, const StateP &lout,
                                               const AdStage &S, const int x[3], idx_t t,
                                               double c, double lf[7])
{
    int l[3] = {x[0], x[1], x[2]};
    l[D] -= 1;
    const idx_t cl = cell_of(g, l);
    // cell update u -= c (F(x + e_D) - F(x))
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int f = lab_cons(D, q);
        lf[q] = c * (lout.u[f][t] - lout.u[f][cl]);
    }
    // F_D[B_t1] enters the edges E_A, A = D + 2, as -F: at x (weights w3h, w4h)
    // and at x + e_C, C = D + 1 (weights w3l, w4l)
    {
        constexpr int A = (D + 2) % 3, C = (A + 2) % 3;
        double w[8];
        edge_weights<A>(g, S, x, w);
        double acc = -0.25 * (1.0 + w[5] + w[7]) * S.le[A][t];
        int y[3] = {x[0], x[1], x[2]};
        y[C] += 1;
        edge_weights<A>(g, S, y, w);
        acc += -0.25 * (1.0 + w[4] + w[6]) * S.le[A][cell_of(g, y)];
        lf[5] = acc;
    }
    // F_D[B_t2] enters the edges E_A, A = D + 1, as +F: at x (weights w1h, w2h)
    // and at x + e_B, B = D + 2 (weights w1l, w2l)
    {
        constexpr int A = (D + 1) % 3, B = (A + 1) % 3;
        double w[8];
        edge_weights<A>(g, S, x, w);
        double acc = 0.25 * (1.0 + w[1] + w[3]) * S.le[A][t];
        int y[3] = {x[0], x[1], x[2]};
        y[B] += 1;
        edge_weights<A>(g, S, y, w);
        acc += 0.25 * (1.0 + w[0] + w[2]) * S.le[A][cell_of(g, y)];
        lf[6] = acc;
    }
}

// faces of axis D of the PCM stage: flux cotangents, then HLLD reversed at
// the forward states (the cell primitives).  The cotangents of the face's two
// states are stored per cell and axis (as the high state of the left cell and
// the low state of the right cell) for the next transpose.  A reconstructing
// stage takes k_ad_faces_row (x) and k_ad_faces_march (y, z).  Two waves per
// SIMD (256 registers and a short spill) beat one wave with 280 registers.
template <int D>
__global__ __launch_bounds__(kBlock, 2) void k_ad_faces(Geom g, Prims P, StateP st, StateP lout,
                                                     AdStage S, StateW lacc,
                                                     const double *dt_dev, double factor)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    int x[3];
    cell_coords(g, t, x);
    double lf[7];
    flux_cotangent<D>(g, lout, S, x, t, factor * dt_dev[0] / g.dl[D], lf);
    auto at = [&](int off) {
        int q[3] = {x[0], x[1], x[2]};
        q[D] += off;
        return pidx(g, q[0], q[1], q[2]);
    };
    const W7 wl = w7_at(P, D, at(-1));
    const W7 wr = w7_at(P, D, at(0));
    const idx_t fo = face_store(g, D, x[0], x[1], x[2]);
    W7 aL{0, 0, 0, 0, 0, 0, 0}, aR{0, 0, 0, 0, 0, 0, 0};
    double abn = 0.0;
    hlld_rev(wl, wr, st.b[D][fo], g.gamma, g.gm1i, lf, aL, aR, abn);
    lacc.b[D][fo] += abn;
    int l[3] = {x[0], x[1], x[2]};
    l[D] -= 1;
    const idx_t cl = cell_of(g, l);
    const double vl[7] = {aL.d, aL.u, aL.v, aL.w, aL.p, aL.by, aL.bz};
    const double vr[7] = {aR.d, aR.u, aR.v, aR.w, aR.p, aR.by, aR.bz};
#pragma unroll
    for (int s = 0; s < 7; ++s) {
        S.lrec[D][7 + s][cl] = vl[s];  // high face of the left cell
        S.lrec[D][s][t] = vr[s];       // low face of the right cell
    }
}

// faces of axis D = y or z with a reconstructing corrector, one thread per
// column (i, j or k) and segment of kAdMarch cells along D: each cell is
// reconstructed once and its high-face state carried to the next face.  Per
// face the same work as k_ad_faces_row.
constexpr int kAdMarch = 16;

__host__ __device__ __forceinline__ idx_t ad_march_blocks(const Geom &g, int D,
                                                          int m = kAdMarch)
{
    const int T = D == 1 ? 2 : 1;
    const idx_t cols = (idx_t)g.n[0] * g.n[T];
    return ((cols + kBlock - 1) / kBlock) * ((g.n[D] + m - 1) / m);
}

// segment of the fused adjoint marches: 16 cells, or 8 on a grid whose
// 16-cell launch would have fewer than 256 blocks (64^3 adjoint 0.93 -> 0.74
// ms; 128^3, 512 blocks, is faster with 16)
static int ad_march_segment(const Geom &g, int D)
{
    const int o = tile_override("admarch");
    if (o == 8 || o == kAdMarch) return o;
    return ad_march_blocks(g, D, kAdMarch) < 256 ? 8 : kAdMarch;
}

template <int D, int RECON>
__global__ __launch_bounds__(kBlock) void k_ad_faces_march(Geom g, Prims P, StateP st,
                                                           StateP lout, AdStage S,
                                                           StateW lacc, const double *dt_dev,
                                                           double factor)
{
    static_assert(D == 1 || D == 2, "columns march along y or z");
    constexpr int T = D == 1 ? 2 : 1;
    constexpr bool kPpm = RECON == VLCT_RECON_PPMC || RECON == VLCT_RECON_PPMP;
    constexpr bool kChar = RECON == VLCT_RECON_PLMC || RECON == VLCT_RECON_PPMC;
    constexpr int R = kPpm ? 2 : 1;
    const int nD = g.n[D];
    const idx_t cols = (idx_t)g.n[0] * g.n[T];
    const idx_t ncb = (cols + kBlock - 1) / kBlock;
    const idx_t b = blockIdx.x;
    const int seg = (int)(b / ncb);
    const idx_t col = (b - (idx_t)seg * ncb) * kBlock + threadIdx.x;
    if (col >= cols) return;
    int x[3];
    x[0] = (int)(col % g.n[0]);
    x[T] = (int)(col / g.n[0]);
    const int s0 = seg * kAdMarch, s1 = min(s0 + kAdMarch, nD);  // cells [s0, s1)
    const double c = factor * dt_dev[0] / g.dl[D];
    auto pid = [&](int along) {
        int q[3] = {x[0], x[1], x[2]};
        q[D] = along;
        return pidx(g, q[0], q[1], q[2]);
    };
    // stencil window of cells a - R .. a + R for a = s0 - 1
    W7 win[2 * R + 1];
    double bnc[2 * R + 1];
#pragma unroll
    for (int q = 0; q < 2 * R + 1; ++q) {
        const idx_t o = pid(s0 - 1 - R + q);
        win[q] = w7_at(P, D, o);
        bnc[q] = P.w[5 + D][o];
    }
    W7 prev{};
    uint32_t fprev = 0;
    for (int a = s0 - 1; a < s1; ++a) {
        W7 fm, fp;
        if constexpr (kPpm)
            ppmc<kChar>(win[0], win[1], win[2], win[3], win[4], bnc[2], g.gamma, fm, fp);
        else
            plmc<kChar>(win[0], win[1], win[2], bnc[1], g.gamma, fm, fp);
        const uint32_t flo = floor_state(fm), fhi = floor_state(fp);
        if (a >= s0) {
            // the face a - 1/2 between the carried high state and this low state
            x[D] = a;
            const idx_t t = cell_of(g, x);
            double lf[7];
            flux_cotangent<D>(g, lout, S, x, t, c, lf);
            const idx_t fo = face_store(g, D, x[0], x[1], x[2]);
            W7 aL{0, 0, 0, 0, 0, 0, 0}, aR{0, 0, 0, 0, 0, 0, 0};
            double abn = 0.0;
            hlld_rev(prev, fm, st.b[D][fo], g.gamma, g.gm1i, lf, aL, aR, abn);
            lacc.b[D][fo] += abn;
            int l[3] = {x[0], x[1], x[2]};
            l[D] -= 1;
            const idx_t cl = cell_of(g, l);
            const double vl[7] = {aL.d, aL.u, aL.v, aL.w, aL.p, aL.by, aL.bz};
            const double vr[7] = {aR.d, aR.u, aR.v, aR.w, aR.p, aR.by, aR.bz};
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                double u = vl[q], v = vr[q];
                if (q == 0 && (fprev & kStatusDensityFloor)) u = 0.0;
                if (q == 4 && (fprev & kStatusPressureFloor)) u = 0.0;
                if (q == 0 && (flo & kStatusDensityFloor)) v = 0.0;
                if (q == 4 && (flo & kStatusPressureFloor)) v = 0.0;
                S.lrec[D][7 + q][cl] = u;  // high face of the cell below
                S.lrec[D][q][t] = v;       // low face of this cell
            }
        }
        prev = fp;
        fprev = fhi;
        if (a + 1 < s1) {
#pragma unroll
            for (int q = 0; q < 2 * R; ++q) {
                win[q] = win[q + 1];
                bnc[q] = bnc[q + 1];
            }
            const idx_t o = pid(a + 1 + R);
            win[2 * R] = w7_at(P, D, o);
            bnc[2 * R] = P.w[5 + D][o];
        }
    }
}

// faces of axis x with a reconstructing corrector: items (row, cell) with
// cells -1 .. nx-1 of every row in one flat sequence; a block reconstructs
// kBlock consecutive items once each, hands the high-face states to the right
// neighbour through LDS, and each item with a left neighbour in its block and
// row takes the face between them (consecutive blocks overlap by one item).
// Per face: flux cotangents, HLLD reversed, the cotangents of the two floored
// states stored per cell and axis (a floored component carries none).
__host__ __device__ __forceinline__ idx_t ad_row_blocks(const Geom &g)
{
    const idx_t items = (idx_t)(g.n[0] + 1) * g.n[1] * g.n[2];
    return (items - 1 + kBlock - 2) / (kBlock - 1);
}

template <int RECON>
__global__ __launch_bounds__(kBlock, 2) void k_ad_faces_row(Geom g, Prims P, StateP st,
                                                         StateP lout, AdStage S, StateW lacc,
                                                         const double *dt_dev, double factor)
{
    constexpr bool kPpm = RECON == VLCT_RECON_PPMC || RECON == VLCT_RECON_PPMP;
    constexpr bool kChar = RECON == VLCT_RECON_PLMC || RECON == VLCT_RECON_PPMC;
    __shared__ double lds[7][kBlock];
    __shared__ uint32_t lfl[kBlock];
    const int nx = g.n[0];
    const idx_t per_row = nx + 1;
    const idx_t items = per_row * g.n[1] * g.n[2];
    const int t = threadIdx.x;
    const idx_t q = (idx_t)blockIdx.x * (kBlock - 1) + t;
    const bool have = q < items;
    const idx_t row = q / per_row;
    int x[3];
    x[0] = (int)(q - row * per_row) - 1;
    x[1] = (int)(row % g.n[1]);
    x[2] = (int)(row / g.n[1]);
    W7 fm{}, fp{};
    uint32_t flo = 0, fhi = 0;
    if (have) {
        auto at = [&](int off) { return pidx(g, x[0] + off, x[1], x[2]); };
        const double bn = P.w[5][at(0)];
        if constexpr (kPpm)
            ppmc<kChar>(w7_at(P, 0, at(-2)), w7_at(P, 0, at(-1)), w7_at(P, 0, at(0)),
                        w7_at(P, 0, at(1)), w7_at(P, 0, at(2)), bn, g.gamma, fm, fp);
        else
            plmc<kChar>(w7_at(P, 0, at(-1)), w7_at(P, 0, at(0)), w7_at(P, 0, at(1)), bn,
                        g.gamma, fm, fp);
        flo = floor_state(fm);
        fhi = floor_state(fp);
    }
    lds[0][t] = fp.d; lds[1][t] = fp.u; lds[2][t] = fp.v; lds[3][t] = fp.w;
    lds[4][t] = fp.p; lds[5][t] = fp.by; lds[6][t] = fp.bz;
    lfl[t] = fhi;
    __syncthreads();
    if (t < 1 || !have || x[0] < 0) return;
    const W7 wl{lds[0][t - 1], lds[1][t - 1], lds[2][t - 1], lds[3][t - 1],
                lds[4][t - 1], lds[5][t - 1], lds[6][t - 1]};
    const uint32_t fl = lfl[t - 1];
    const idx_t tc = cell_of(g, x);
    double lf[7];
    flux_cotangent<0>(g, lout, S, x, tc, factor * dt_dev[0] / g.dl[0], lf);
    const idx_t fo = face_store(g, 0, x[0], x[1], x[2]);
    W7 aL{0, 0, 0, 0, 0, 0, 0}, aR{0, 0, 0, 0, 0, 0, 0};
    double abn = 0.0;
    hlld_rev(wl, fm, st.b[0][fo], g.gamma, g.gm1i, lf, aL, aR, abn);
    lacc.b[0][fo] += abn;
    const idx_t cl = cell_of(g, x[0] - 1, x[1], x[2]);
    const double vl[7] = {aL.d, aL.u, aL.v, aL.w, aL.p, aL.by, aL.bz};
    const double vr[7] = {aR.d, aR.u, aR.v, aR.w, aR.p, aR.by, aR.bz};
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        double u = vl[c], v = vr[c];
        if (c == 0 && (fl & kStatusDensityFloor)) u = 0.0;
        if (c == 4 && (fl & kStatusPressureFloor)) u = 0.0;
        if (c == 0 && (flo & kStatusDensityFloor)) v = 0.0;
        if (c == 4 && (flo & kStatusPressureFloor)) v = 0.0;
        S.lrec[0][7 + c][cl] = u;  // high face of the left cell
        S.lrec[0][c][tc] = v;      // low face of this cell
    }
}

// y and z faces of a linear-reconstruction stage with the reconstruction
// transposed in the same march: a segment computes its faces and the one
// above it (whose cotangent the top cell needs; its normal-field cotangent
// stays with the segment that owns it), and as soon as a cell has the
// cotangents of both its interface states it reverses its reconstruction.
template <int D, int RECON, int M = kAdMarch>
__global__ __launch_bounds__(kBlock) void k_ad_march_fused(Geom g, Prims P, StateP st,
                                                           StateP lout, AdStage S,
                                                           StateW lacc, const double *dt_dev,
                                                           double factor)
{
    static_assert(D == 1 || D == 2, "columns march along y or z");
    static_assert(RECON == VLCT_RECON_PLMC || RECON == VLCT_RECON_PLMP, "linear reconstructions");
    constexpr int T = D == 1 ? 2 : 1;
    constexpr bool kChar = RECON == VLCT_RECON_PLMC;
    const int nD = g.n[D];
    const idx_t cols = (idx_t)g.n[0] * g.n[T];
    const idx_t ncb = (cols + kBlock - 1) / kBlock;
    const idx_t b = blockIdx.x;
    const int seg = (int)(b / ncb);
    const idx_t col = (b - (idx_t)seg * ncb) * kBlock + threadIdx.x;
    if (col >= cols) return;
    int x[3];
    x[0] = (int)(col % g.n[0]);
    x[T] = (int)(col / g.n[0]);
    const int s0 = seg * M, s1 = min(s0 + M, nD);  // cells [s0, s1)
    const double c = factor * dt_dev[0] / g.dl[D];
    auto pid = [&](int along) {
        int q[3] = {x[0], x[1], x[2]};
        q[D] = along;
        return pidx(g, q[0], q[1], q[2]);
    };
    // window of cells a - 2 .. a + 1 for the cell a being reconstructed
    W7 win[4];
    double bnc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const idx_t o = pid(s0 - 3 + q);
        win[q] = w7_at(P, D, o);
        bnc[q] = P.w[5 + D][o];
    }
    W7 prev{};
    uint32_t fprev = 0;
    double alow[7];  // cotangent of the low-face state of the cell below the face
    // the reversal of cell m adds to the cells m - 1, m and m + 1, after which
    // cell m - 1 has all its terms from this segment: the cells m and m + 1
    // wait in LDS (cell c in slot c & 1, each thread its own column) and a
    // cell leaves with one atomic add per component (segments share the two
    // cells at each end)
    __shared__ double pend[2][7][kBlock];
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        pend[0][k][tid] = 0.0;
        pend[1][k][tid] = 0.0;
    }
    for (int a = s0 - 1; a <= s1; ++a) {
        W7 fm, fp;
        plmc<kChar>(win[1], win[2], win[3], bnc[2], g.gamma, fm, fp);
        const uint32_t flo = floor_state(fm), fhi = floor_state(fp);
        if (a >= s0) {
            // the face a - 1/2
            x[D] = a;
            const idx_t t = cell_of(g, x);
            double lf[7];
            flux_cotangent<D>(g, lout, S, x, t, c, lf);
            int m[3] = {x[0], x[1], x[2]};
            m[D] = wrapc(a, nD);
            const idx_t fo = face_store(g, D, m[0], m[1], m[2]);
            W7 aL{0, 0, 0, 0, 0, 0, 0}, aR{0, 0, 0, 0, 0, 0, 0};
            double abn = 0.0;
            hlld_rev(prev, fm, st.b[D][fo], g.gamma, g.gm1i, lf, aL, aR, abn);
            if (a < s1) lacc.b[D][fo] += abn;
            double ahigh[7] = {aL.d, aL.u, aL.v, aL.w, aL.p, aL.by, aL.bz};
            if (fprev & kStatusDensityFloor) ahigh[0] = 0.0;
            if (fprev & kStatusPressureFloor) ahigh[4] = 0.0;
            if (a - 1 >= s0) {
                // cell a - 1 has both interface cotangents: reverse its PLM
                W7 am{0, 0, 0, 0, 0, 0, 0}, a0{0, 0, 0, 0, 0, 0, 0}, ap{0, 0, 0, 0, 0, 0, 0};
                double abc = 0.0;
                plmc_rev<kChar>(win[0], win[1], win[2], bnc[1], g.gamma, alow, ahigh, am, a0,
                                ap, abc);
                const double vm[7] = {am.d, am.u, am.v, am.w, am.p, am.by, am.bz};
                const double v0[7] = {a0.d, a0.u, a0.v, a0.w, a0.p, a0.by, a0.bz};
                const double vp[7] = {ap.d, ap.u, ap.v, ap.w, ap.p, ap.by, ap.bz};
                const int so = (a - 2) & 1, sn = (a - 1) & 1;  // slots of cells a - 2 (and a), a - 1
                int e[3] = {x[0], x[1], x[2]};
                e[D] = a - 2;
                const idx_t cm = cell_of(g, e);
#pragma unroll
                for (int k = 0; k < 7; ++k) {
                    atomicAdd(&S.lw[lab_slot(D, k)][cm], pend[so][k][tid] + vm[k]);
                    pend[so][k][tid] = vp[k];
                    pend[sn][k][tid] += v0[k];
                }
                e[D] = a - 1;
                atomicAdd(&S.lw[5 + D][cell_of(g, e)], abc);
            }
            const double lo[7] = {aR.d, aR.u, aR.v, aR.w, aR.p, aR.by, aR.bz};
#pragma unroll
            for (int k = 0; k < 7; ++k) alow[k] = lo[k];
            if (flo & kStatusDensityFloor) alow[0] = 0.0;
            if (flo & kStatusPressureFloor) alow[4] = 0.0;
        }
        prev = fp;
        fprev = fhi;
        if (a + 1 <= s1) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                win[q] = win[q + 1];
                bnc[q] = bnc[q + 1];
            }
            const idx_t o = pid(a + 2);
            win[3] = w7_at(P, D, o);
            bnc[3] = P.w[5 + D][o];
        }
    }
    // the cells s1 - 1 and s1 (the last reversal was that of cell s1 - 1)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        int e[3] = {x[0], x[1], x[2]};
        e[D] = s1 - 1 + q;
        const idx_t cc = cell_of(g, e);
        const int sl = (s1 - 1 + q) & 1;
#pragma unroll
        for (int k = 0; k < 7; ++k) atomicAdd(&S.lw[lab_slot(D, k)][cc], pend[sl][k][tid]);
    }
}

// x faces of a linear-reconstruction stage with the reconstruction transposed
// in the same kernel: items (row, cell) with cells -1 .. nx of every row in
// one flat sequence, blocks of kBlock items overlapping by two.  Each item
// reconstructs its cell and hands the high-face state to the right through
// LDS; each item with a left neighbour in its block and row takes the face
// between them and hands the left state's cotangent back; each item whose
// faces both lie in the block and which is a cell of the grid then reverses
// its reconstruction.  A face computed twice (the last of a block, the
// periodic image at the end of a row) leaves its normal-field cotangent to
// the item that owns it.
__host__ __device__ __forceinline__ idx_t ad_row_fused_blocks(const Geom &g)
{
    const idx_t items = (idx_t)(g.n[0] + 2) * g.n[1] * g.n[2];
    return (items - 1 + kBlock - 3) / (kBlock - 2);  // items 1 .. items-1 at t in [1, kBlock-2]
}

template <int RECON>
__global__ __launch_bounds__(kBlock) void k_ad_row_fused(Geom g, Prims P, StateP st,
                                                         StateP lout, AdStage S, StateW lacc,
                                                         const double *dt_dev, double factor)
{
    static_assert(RECON == VLCT_RECON_PLMC || RECON == VLCT_RECON_PLMP, "linear reconstructions");
    constexpr bool kChar = RECON == VLCT_RECON_PLMC;
    __shared__ double lds[7][kBlock];
    __shared__ double lds_p[7][kBlock];
    __shared__ uint32_t lfl[kBlock];
    __shared__ uint32_t lrev[kBlock];
    const int nx = g.n[0];
    const idx_t per_row = nx + 2;
    const idx_t items = per_row * g.n[1] * g.n[2];
    const int t = threadIdx.x;
    const idx_t q = (idx_t)blockIdx.x * (kBlock - 2) + t;
    const bool have = q < items;
    const idx_t row = q / per_row;
    int x[3];
    x[0] = (int)(q - row * per_row) - 1;
    x[1] = (int)(row % g.n[1]);
    x[2] = (int)(row / g.n[1]);
    auto at = [&](int off) { return pidx(g, x[0] + off, x[1], x[2]); };
    W7 fm{}, fp{};
    uint32_t flo = 0, fhi = 0;
    if (have) {
        plmc<kChar>(w7_at(P, 0, at(-1)), w7_at(P, 0, at(0)), w7_at(P, 0, at(1)),
                    P.w[5][at(0)], g.gamma, fm, fp);
        flo = floor_state(fm);
        fhi = floor_state(fp);
    }
    lds[0][t] = fp.d; lds[1][t] = fp.u; lds[2][t] = fp.v; lds[3][t] = fp.w;
    lds[4][t] = fp.p; lds[5][t] = fp.by; lds[6][t] = fp.bz;
    lfl[t] = fhi;
    __syncthreads();
    // the face x - 1/2 (x in 0 .. nx), between the item on the left and this one
    const bool face = t >= 1 && have && x[0] >= 0;
    double alow[7] = {0, 0, 0, 0, 0, 0, 0}, ahigh_left[7] = {0, 0, 0, 0, 0, 0, 0};
    if (face) {
        const W7 wl{lds[0][t - 1], lds[1][t - 1], lds[2][t - 1], lds[3][t - 1],
                    lds[4][t - 1], lds[5][t - 1], lds[6][t - 1]};
        const uint32_t fl = lfl[t - 1];
        const idx_t tc = cell_of(g, x);
        double lf[7];
        flux_cotangent<0>(g, lout, S, x, tc, factor * dt_dev[0] / g.dl[0], lf);
        const idx_t fo = face_store(g, 0, wrapc(x[0], nx), x[1], x[2]);
        W7 aL{0, 0, 0, 0, 0, 0, 0}, aR{0, 0, 0, 0, 0, 0, 0};
        double abn = 0.0;
        hlld_rev(wl, fm, st.b[0][fo], g.gamma, g.gm1i, lf, aL, aR, abn);
        if (t <= kBlock - 2 && x[0] < nx) lacc.b[0][fo] += abn;
        const double vl[7] = {aL.d, aL.u, aL.v, aL.w, aL.p, aL.by, aL.bz};
        const double vr[7] = {aR.d, aR.u, aR.v, aR.w, aR.p, aR.by, aR.bz};
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            ahigh_left[c] = vl[c];
            alow[c] = vr[c];
        }
        if (fl & kStatusDensityFloor) ahigh_left[0] = 0.0;
        if (fl & kStatusPressureFloor) ahigh_left[4] = 0.0;
        if (flo & kStatusDensityFloor) alow[0] = 0.0;
        if (flo & kStatusPressureFloor) alow[4] = 0.0;
    }
    __syncthreads();
    // hand the left state's cotangent to the item on the left
#pragma unroll
    for (int c = 0; c < 7; ++c) lds[c][t] = ahigh_left[c];
    __syncthreads();
    const bool rev = face && t <= kBlock - 2 && x[0] < nx;
    W7 am{0, 0, 0, 0, 0, 0, 0}, a0{0, 0, 0, 0, 0, 0, 0}, ap{0, 0, 0, 0, 0, 0, 0};
    double abc = 0.0;
    if (rev) {
        double ahigh[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) ahigh[c] = lds[c][t + 1];
        plmc_rev<kChar>(w7_at(P, 0, at(-1)), w7_at(P, 0, at(0)), w7_at(P, 0, at(1)),
                        P.w[5][at(0)], g.gamma, alow, ahigh, am, a0, ap, abc);
    }
    __syncthreads();
    // the reversal adds to the cells x - 1, x and x + 1: the neighbours' terms
    // go through LDS to the item that owns the cell where it reversed too, so
    // that each cell leaves with one atomic add per component
    const double vm[7] = {am.d, am.u, am.v, am.w, am.p, am.by, am.bz};
    const double vp[7] = {ap.d, ap.u, ap.v, ap.w, ap.p, ap.by, ap.bz};
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        lds[c][t] = vm[c];
        lds_p[c][t] = vp[c];
    }
    lrev[t] = rev ? 1u : 0u;
    __syncthreads();
    if (!rev) return;
    // an item that reversed on the left (right) is the cell x - 1 (x + 1) of this row
    const bool left_rev = t >= 1 && lrev[t - 1];
    const bool right_rev = lrev[t + 1] != 0u;
    const double v0[7] = {a0.d, a0.u, a0.v, a0.w, a0.p, a0.by, a0.bz};
    const idx_t cc = cell_of(g, x);
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        double v = v0[c];
        if (left_rev) v += lds_p[c][t - 1];
        if (right_rev) v += lds[c][t + 1];
        atomicAdd(&S.lw[lab_slot(0, c)][cc], v);
    }
    if (!left_rev) {
        const idx_t cl = cell_of(g, x[0] - 1, x[1], x[2]);
#pragma unroll
        for (int c = 0; c < 7; ++c) atomicAdd(&S.lw[lab_slot(0, c)][cl], vm[c]);
    }
    if (!right_rev) {
        const idx_t cr = cell_of(g, x[0] + 1, x[1], x[2]);
#pragma unroll
        for (int c = 0; c < 7; ++c) atomicAdd(&S.lw[lab_slot(0, c)][cr], vp[c]);
    }
    atomicAdd(&S.lw[5][cc], abc);
}

// reconstruction of each cell along D reversed: cotangents of the stencil
// states (three cells for PLM, five for PPM) and of the cell's B_cc,D
template <int D, int RECON>
__global__ __launch_bounds__(kBlock) void k_ad_recon(Geom g, Prims P, AdStage S)
{
    constexpr bool kPpm = RECON == VLCT_RECON_PPMC || RECON == VLCT_RECON_PPMP;
    constexpr bool kChar = RECON == VLCT_RECON_PLMC || RECON == VLCT_RECON_PPMC;
    constexpr int kR = kPpm ? 2 : 1;  // stencil radius
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    int x[3];
    cell_coords(g, t, x);
    double afm[7], afp[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        afm[c] = S.lrec[D][c][t];
        afp[c] = S.lrec[D][7 + c][t];
    }
    idx_t po[2 * kR + 1];
#pragma unroll
    for (int q = 0; q <= 2 * kR; ++q) {
        int e[3] = {x[0], x[1], x[2]};
        e[D] += q - kR;
        po[q] = pidx(g, e[0], e[1], e[2]);
    }
    W7 ad[2 * kR + 1];
#pragma unroll
    for (int q = 0; q <= 2 * kR; ++q) ad[q] = W7{0, 0, 0, 0, 0, 0, 0};
    double abn = 0.0;
    if (kPpm) {
        ppmc_rev<kChar>(w7_at(P, D, po[0]), w7_at(P, D, po[1]), w7_at(P, D, po[kR]),
                        w7_at(P, D, po[2 * kR - 1]), w7_at(P, D, po[2 * kR]),
                        P.w[5 + D][po[kR]], g.gamma, afm, afp, ad[0], ad[1], ad[kR],
                        ad[2 * kR - 1], ad[2 * kR], abn);
    } else {
        plmc_rev<kChar>(w7_at(P, D, po[0]), w7_at(P, D, po[1]), w7_at(P, D, po[2]),
                        P.w[5 + D][po[1]], g.gamma, afm, afp, ad[0], ad[1], ad[2], abn);
    }
#pragma unroll
    for (int q = 0; q <= 2 * kR; ++q) {
        int e[3] = {x[0], x[1], x[2]};
        e[D] += q - kR;
        const idx_t c = cell_of(g, e);
        const W7 &v = ad[q];
        const double a[7] = {v.d, v.u, v.v, v.w, v.p, v.by, v.bz};
#pragma unroll
        for (int s = 0; s < 7; ++s) atomicAdd(&S.lw[lab_slot(D, s)][c], a[s]);
    }
    atomicAdd(&S.lw[5 + D][t], abn);
}

// The parabolic reversals add each cell's stencil cotangents (five cells)
// without one atomic per term.  Along y and z a thread marches a column
// segment of M cells and keeps the four cells still waiting for terms in LDS
// (thread-private slots, cell c in slot c mod 5); a cell leaves with one
// atomic add per component once the reversal two cells above it is done
// (segments share two cells at each end, so every departure stays atomic).
// The cell's own B_n cotangent comes from its reversal alone and is added
// in place.
template <int D, int RECON, int M = kAdMarch>
__global__ __launch_bounds__(kBlock) void k_ad_recon_march(Geom g, Prims P, AdStage S)
{
    static_assert(D == 1 || D == 2, "columns march along y or z");
    static_assert(RECON == VLCT_RECON_PPMC || RECON == VLCT_RECON_PPMP, "parabolic reconstructions");
    constexpr int T = D == 1 ? 2 : 1;
    constexpr bool kChar = RECON == VLCT_RECON_PPMC;
    __shared__ double pend[5][7][kBlock];
    const int nD = g.n[D];
    const idx_t cols = (idx_t)g.n[0] * g.n[T];
    const idx_t ncb = (cols + kBlock - 1) / kBlock;
    const idx_t b = blockIdx.x;
    const int seg = (int)(b / ncb);
    const idx_t col = (b - (idx_t)seg * ncb) * kBlock + threadIdx.x;
    if (col >= cols) return;
    const int tid = threadIdx.x;
    int x[3];
    x[0] = (int)(col % g.n[0]);
    x[T] = (int)(col / g.n[0]);
    const int s0 = seg * M, s1 = min(s0 + M, nD);  // cells [s0, s1)
    auto slot = [](int c) { return (c + 10) % 5; };  // c >= -2
    auto cell_at = [&](int along) {
        int e[3] = {x[0], x[1], x[2]};
        e[D] = along;
        return cell_of(g, e);
    };
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 7; ++k) pend[slot(s0 - 2 + q)][k][tid] = 0.0;
    for (int c = s0; c < s1; ++c) {
        const idx_t t = cell_at(c);
        double afm[7], afp[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            afm[k] = S.lrec[D][k][t];
            afp[k] = S.lrec[D][7 + k][t];
        }
        idx_t po[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            int e[3] = {x[0], x[1], x[2]};
            e[D] = c - 2 + q;
            po[q] = pidx(g, e[0], e[1], e[2]);
        }
        W7 ad[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) ad[q] = W7{0, 0, 0, 0, 0, 0, 0};
        double abn = 0.0;
        ppmc_rev<kChar>(w7_at(P, D, po[0]), w7_at(P, D, po[1]), w7_at(P, D, po[2]),
                        w7_at(P, D, po[3]), w7_at(P, D, po[4]), P.w[5 + D][po[2]], g.gamma,
                        afm, afp, ad[0], ad[1], ad[2], ad[3], ad[4], abn);
        double v[5][7];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            v[q][0] = ad[q].d; v[q][1] = ad[q].u; v[q][2] = ad[q].v; v[q][3] = ad[q].w;
            v[q][4] = ad[q].p; v[q][5] = ad[q].by; v[q][6] = ad[q].bz;
        }
        const idx_t cm = cell_at(c - 2);
        const int sm = slot(c - 2), s1m = slot(c - 1), s00 = slot(c), s1p = slot(c + 1),
                  s2p = slot(c + 2);
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            atomicAdd(&S.lw[lab_slot(D, k)][cm], pend[sm][k][tid] + v[0][k]);
            pend[s1m][k][tid] += v[1][k];
            pend[s00][k][tid] += v[2][k];
            pend[s1p][k][tid] += v[3][k];
            pend[s2p][k][tid] = v[4][k];
        }
        S.lw[5 + D][t] += abn;
    }
    // the cells s1 - 2 .. s1 + 1 (the last reversal was that of cell s1 - 1)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const idx_t cc = cell_at(s1 - 2 + q);
        const int sl = slot(s1 - 2 + q);
#pragma unroll
        for (int k = 0; k < 7; ++k) atomicAdd(&S.lw[lab_slot(D, k)][cc], pend[sl][k][tid]);
    }
}

// cotangent of -(v x B)_A at cell x from the four A-edges around it
template <int A>
__device__ __forceinline__ double eref_cotangent(const Geom &g, const AdStage &S, const int x[3])
{
    constexpr int B = (A + 1) % 3, C = (A + 2) % 3;
    double w[8], acc;
    // the cell is r00 of edge x, r10 of edge x + e_B, r01 of edge x + e_C and
    // r11 of edge x + e_B + e_C
    edge_weights<A>(g, S, x, w);
    acc = (w[1] + w[5]) * S.le[A][cell_of(g, x)];
    int y[3] = {x[0], x[1], x[2]};
    y[B] += 1;
    edge_weights<A>(g, S, y, w);
    acc += (w[0] + w[7]) * S.le[A][cell_of(g, y)];
    y[B] -= 1;
    y[C] += 1;
    edge_weights<A>(g, S, y, w);
    acc += (w[3] + w[4]) * S.le[A][cell_of(g, y)];
    y[B] += 1;
    edge_weights<A>(g, S, y, w);
    acc += (w[2] + w[6]) * S.le[A][cell_of(g, y)];
    return -0.25 * acc;
}

// reference fields -(v x B) and primitive recovery (Sec. 2.1; B_cc = face
// average) reversed into the cotangents of the stage's conserved cells and
// faces; a floored quantity is a constant.  GATHER (PCM stage): the primitive
// cotangents are the sums of the stored face-state cotangents of the cell;
// otherwise the reconstruction transposes have accumulated them.
template <bool GATHER>
__global__ __launch_bounds__(kBlock) void k_ad_prims(Geom g, StateP st, Prims P, AdStage S, StateW lacc)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    int x[3];
    cell_coords(g, t, x);
    const int i = x[0], j = x[1], k = x[2];
    double lw[8];
    if (GATHER) {
#pragma unroll
        for (int f = 0; f < 8; ++f) lw[f] = 0.0;
#pragma unroll
        for (int D = 0; D < 3; ++D)
#pragma unroll
            for (int q = 0; q < 7; ++q)
                lw[lab_slot(D, q)] += S.lrec[D][q][t] + S.lrec[D][7 + q][t];
    } else {
#pragma unroll
        for (int f = 0; f < 8; ++f) lw[f] = S.lw[f][t];
    }
    {
        const idx_t o = pidx(g, i, j, k);
        const double vx = P.w[1][o], vy = P.w[2][o], vz = P.w[3][o];
        const double bx = P.w[5][o], by = P.w[6][o], bz = P.w[7][o];
        const double ex = eref_cotangent<0>(g, S, x), ey = eref_cotangent<1>(g, S, x),
                     ez = eref_cotangent<2>(g, S, x);
        lw[1] += bz * ey - by * ez;
        lw[2] += -bz * ex + bx * ez;
        lw[3] += by * ex - bx * ey;
        lw[5] += -vz * ey + vy * ez;
        lw[6] += vz * ex - vx * ez;
        lw[7] += -vy * ex + vx * ey;
    }
    const idx_t fl[3] = {face_store(g, 0, i, j, k), face_store(g, 1, i, j, k),
                         face_store(g, 2, i, j, k)};
    const idx_t fh[3] = {face_store(g, 0, wrapc(i + 1, g.n[0]), j, k),
                         face_store(g, 1, i, wrapc(j + 1, g.n[1]), k),
                         face_store(g, 2, i, j, wrapc(k + 1, g.n[2]))};
    double bc[3];
    for (int d = 0; d < 3; ++d) bc[d] = 0.5 * (st.b[d][fl[d]] + st.b[d][fh[d]]);
    double d = st.u[0][t];
    const bool dfloor = !(d >= kFloorRho);
    if (dfloor) d = kFloorRho;
    const double id = 1.0 / d;
    const double v[3] = {st.u[1][t] * id, st.u[2][t] * id, st.u[3][t] * id};
    const double ke = 0.5 * d * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double me = 0.5 * (bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
    const double p = (g.gamma - 1.0) * (st.u[4][t] - ke - me);
    const bool pfloor = !(p >= kFloorP);
    const double gm1 = g.gamma - 1.0;
    const double lp = pfloor ? 0.0 : lw[4];
    const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double lrho = dfloor ? 0.0 : lw[0] + lp * gm1 * 0.5 * v2;
    for (int l = 0; l < 3; ++l) {
        if (!dfloor) lrho -= lw[1 + l] * v[l] * id;
        lacc.u[1 + l][t] += lw[1 + l] * id - lp * gm1 * v[l];
    }
    lacc.u[0][t] += lrho;
    lacc.u[4][t] += lp * gm1;
    for (int l = 0; l < 3; ++l) {
        const double lb = 0.5 * (lw[5 + l] - lp * gm1 * bc[l]);
        atomicAdd(&lacc.b[l][fl[l]], lb);
        atomicAdd(&lacc.b[l][fh[l]], lb);
    }
}

// transposes of one stage: lout is the cotangent of the stage's output state,
// st/P/sd the stage's input state, primitives and upwind sides; the result
// is added to lacc (the cotangent of the stage's input state).
static void stage_adjoint(const Geom &g, double factor, const StateP &lout, const StateP &st,
                          const Prims &P, const Sides &sd, int recon, const AdStage &S,
                          const StateW &lacc, const double *dt, hipStream_t s)
{
    const unsigned gc = nblocks((size_t)g.n[0] * g.n[1] * g.n[2]);
    k_ad_edges<<<gc, kBlock, 0, s>>>(g, lout, sd, S, dt, factor, recon != VLCT_RECON_PCM);
#define VLCT_AD_FACES(R)                                                             \
    k_ad_faces_row<R><<<(unsigned)ad_row_blocks(g), kBlock, 0, s>>>(g, P, st, lout, S,     \
                                                                     lacc, dt, factor);    \
    k_ad_faces_march<1, R><<<(unsigned)ad_march_blocks(g, 1), kBlock, 0, s>>>(             \
        g, P, st, lout, S, lacc, dt, factor);                                              \
    k_ad_faces_march<2, R><<<(unsigned)ad_march_blocks(g, 2), kBlock, 0, s>>>(             \
        g, P, st, lout, S, lacc, dt, factor);
#define VLCT_AD_FUSED(R)                                                                   \
    k_ad_row_fused<R><<<(unsigned)ad_row_fused_blocks(g), kBlock, 0, s>>>(g, P, st, lout,  \
                                                                           S, lacc, dt,    \
                                                                           factor);        \
    if (ad_march_segment(g, 1) == 8)                                                       \
        k_ad_march_fused<1, R, 8><<<(unsigned)ad_march_blocks(g, 1, 8), kBlock, 0, s>>>(   \
            g, P, st, lout, S, lacc, dt, factor);                                          \
    else                                                                                   \
        k_ad_march_fused<1, R><<<(unsigned)ad_march_blocks(g, 1), kBlock, 0, s>>>(         \
            g, P, st, lout, S, lacc, dt, factor);                                          \
    if (ad_march_segment(g, 2) == 8)                                                       \
        k_ad_march_fused<2, R, 8><<<(unsigned)ad_march_blocks(g, 2, 8), kBlock, 0, s>>>(   \
            g, P, st, lout, S, lacc, dt, factor);                                          \
    else                                                                                   \
        k_ad_march_fused<2, R><<<(unsigned)ad_march_blocks(g, 2), kBlock, 0, s>>>(         \
            g, P, st, lout, S, lacc, dt, factor);
#define VLCT_AD_RECON(R)                                                                   \
    k_ad_recon<0, R><<<gc, kBlock, 0, s>>>(g, P, S);                                       \
    if (ad_march_segment(g, 1) == 8)                                                       \
        k_ad_recon_march<1, R, 8><<<(unsigned)ad_march_blocks(g, 1, 8), kBlock, 0, s>>>(g, P, S); \
    else                                                                                   \
        k_ad_recon_march<1, R><<<(unsigned)ad_march_blocks(g, 1), kBlock, 0, s>>>(g, P, S); \
    if (ad_march_segment(g, 2) == 8)                                                       \
        k_ad_recon_march<2, R, 8><<<(unsigned)ad_march_blocks(g, 2, 8), kBlock, 0, s>>>(g, P, S); \
    else                                                                                   \
        k_ad_recon_march<2, R><<<(unsigned)ad_march_blocks(g, 2), kBlock, 0, s>>>(g, P, S);
    if (recon == VLCT_RECON_PCM) {
        k_ad_faces<0><<<gc, kBlock, 0, s>>>(g, P, st, lout, S, lacc, dt, factor);
        k_ad_faces<1><<<gc, kBlock, 0, s>>>(g, P, st, lout, S, lacc, dt, factor);
        k_ad_faces<2><<<gc, kBlock, 0, s>>>(g, P, st, lout, S, lacc, dt, factor);
    } else if (recon == VLCT_RECON_PLMC) {
        VLCT_AD_FUSED(VLCT_RECON_PLMC)
    } else if (recon == VLCT_RECON_PLMP) {
        VLCT_AD_FUSED(VLCT_RECON_PLMP)
    } else if (recon == VLCT_RECON_PPMC) {
        VLCT_AD_FACES(VLCT_RECON_PPMC)
        VLCT_AD_RECON(VLCT_RECON_PPMC)
    } else {
        VLCT_AD_FACES(VLCT_RECON_PPMP)
        VLCT_AD_RECON(VLCT_RECON_PPMP)
    }
#undef VLCT_AD_FACES
#undef VLCT_AD_FUSED
#undef VLCT_AD_RECON
    if (recon == VLCT_RECON_PCM)
        k_ad_prims<true><<<gc, kBlock, 0, s>>>(g, st, P, S, lacc);
    else
        k_ad_prims<false><<<gc, kBlock, 0, s>>>(g, st, P, S, lacc);
}

// workspace of the adjoint: forward intermediates and cotangents.  Without a
// tape it also holds the recomputed fluxes, half-step state and upwind sides.
struct AdLayout {
    size_t prims[2], half[8], flux[2][3], side[2][3], le, wcode, lw, lrec, total;
    size_t prims_len, flux_len[3], cell_pitch;
    size_t lnext[8], lhalf[8];
};

static AdLayout ad_layout(const Geom &g, bool taped)
{
    AdLayout L;
    size_t off = 0;
    const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    L.cell_pitch = align_up(N * 8);
    L.prims_len = (size_t)g.p[0] * g.p[1] * g.p[2];
    for (int h = 0; h < 2; ++h) {
        L.prims[h] = off;
        off += 8 * align_up(L.prims_len * 8);
    }
    for (int d = 0; d < 3; ++d)
        L.flux_len[d] = (size_t)flux_dim(g.n, d, 0) * flux_dim(g.n, d, 1) * flux_dim(g.n, d, 2);
    if (!taped) {
        for (int f = 0; f < 8; ++f) {
            L.half[f] = off;
            off += align_up(field_len(g.n, f) * 8);
        }
        for (int h = 0; h < 2; ++h)
            for (int d = 0; d < 3; ++d) {
                L.flux[h][d] = off;
                off += flux_axis_bytes(L.flux_len[d]);
            }
        for (int h = 0; h < 2; ++h)
            for (int d = 0; d < 3; ++d) {
                L.side[h][d] = off;
                off += align_up(N);
            }
    }
    for (int f = 0; f < 8; ++f) {
        L.lnext[f] = off;
        off += align_up(field_len(g.n, f) * 8);
    }
    for (int f = 0; f < 8; ++f) {
        L.lhalf[f] = off;
        off += align_up(field_len(g.n, f) * 8);
    }
    L.le = off;
    off += 3 * L.cell_pitch;
    L.wcode = off;
    off += align_up(N * sizeof(uint32_t));
    L.lw = off;
    off += 8 * L.cell_pitch;
    L.lrec = off;
    off += 42 * L.cell_pitch;
    L.total = off;
    return L;
}

// argument checks shared by both adjoint entry points
static int adjoint_args(const vlct_grid *vg, const vlct_state *in, const vlct_state *lam_out,
                        const vlct_state *lam_in, const double *dt_dev)
{
    if (!grid_ok(vg) || !state_ok(in) || !state_ok(lam_out) || !state_ok(lam_in) || !dt_dev)
        return VLCT_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (vg->bc[d] != VLCT_BC_PERIODIC) return VLCT_EUNSUPPORTED;
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
    return VLCT_OK;
}

// the adjoint of one step given the half-step state and both stages' upwind
// sides (from a tape, or recomputed into the workspace by the caller, who
// then has also computed both stages' primitives: have_prims)
static int adjoint_core(const vlct_grid *vg, const Geom &g, const AdLayout &L, char *b,
                        const StateP &sin, const StateP &hc, const Sides sides[2],
                        bool have_prims, const vlct_state *lam_out, const vlct_state *lam_in,
                        const double *dt_dev, hipStream_t s)
{
    auto arr = [&](size_t off) { return reinterpret_cast<double *>(b + off); };
    Prims P[2];
    for (int h = 0; h < 2; ++h)
        for (int f = 0; f < 8; ++f) P[h].w[f] = arr(L.prims[h] + f * align_up(L.prims_len * 8));
    StateW lnext, lhalf;
    for (int f = 0; f < 8; ++f) {
        double *c = arr(L.lnext[f]), *e = arr(L.lhalf[f]);
        if (f < 5) { lnext.u[f] = c; lhalf.u[f] = e; }
        else { lnext.b[f - 5] = c; lhalf.b[f - 5] = e; }
    }
    AdStage S;
    for (int a = 0; a < 3; ++a) S.le[a] = arr(L.le + a * L.cell_pitch);
    S.wcode = reinterpret_cast<uint32_t *>(b + L.wcode);
    for (int f = 0; f < 8; ++f) S.lw[f] = arr(L.lw + f * L.cell_pitch);
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 14; ++c) S.lrec[d][c] = arr(L.lrec + (14 * d + c) * L.cell_pitch);

    // primitives of both stages' input states (same kernel as the step)
    if (!have_prims) {
        int rc = launch_prims(g, sin, P[0], nullptr, s);
        if (!rc) rc = launch_prims(g, hc, P[1], nullptr, s);
        if (rc) return rc;
    }

    // reverse: corrector stage into mu = lhalf, then lam_in += mu + predictor^T mu
    const StateW lin = as_mut(lam_in);
    const unsigned gf = nblocks((size_t)(g.n[0] + 1) * (g.n[1] + 1) * (g.n[2] + 1));
    k_ad_init<<<gf, kBlock, 0, s>>>(g, as_const(lam_out), lnext, lhalf);
    stage_adjoint(g, 1.0, as_const(lnext), hc, P[1], sides[1], vg->recon, S, lhalf,
                  dt_dev, s);
    k_ad_add<<<gf, kBlock, 0, s>>>(g, lin, as_const(lnext), as_const(lhalf));
    stage_adjoint(g, 0.5, as_const(lhalf), sin, P[0], sides[0], VLCT_RECON_PCM, S, lin,
                  dt_dev, s);
    return hipGetLastError() == hipSuccess ? VLCT_OK : VLCT_EHIP;
}

// ---------------------------------------------------------------------------
// face fields from an edge-centred vector potential, B = curl_h A (periodic),
// and the transpose of that map.  A_x at (i, j-1/2, k-1/2), A_y at
// (i-1/2, j, k-1/2), A_z at (i-1/2, j-1/2, k), each stored like a cell array.
// ---------------------------------------------------------------------------
__global__ void k_curl_potential(Geom g, const double *ax, const double *ay, const double *az,
                                 double *bx, double *by, double *bz)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    int x[3];
    cell_coords(g, t, x);
    const int i = x[0], j = x[1], k = x[2];
    const idx_t ip = cell_of(g, i + 1, j, k), jp = cell_of(g, i, j + 1, k),
                kp = cell_of(g, i, j, k + 1);
    const double vx = (az[jp] - az[t]) / g.dl[1] - (ay[kp] - ay[t]) / g.dl[2];
    const double vy = (ax[kp] - ax[t]) / g.dl[2] - (az[ip] - az[t]) / g.dl[0];
    const double vz = (ay[ip] - ay[t]) / g.dl[0] - (ax[jp] - ax[t]) / g.dl[1];
    bx[face_store(g, 0, i, j, k)] = vx;
    by[face_store(g, 1, i, j, k)] = vy;
    bz[face_store(g, 2, i, j, k)] = vz;
    // the duplicate periodic face planes
    if (i == 0) bx[face_store(g, 0, g.n[0], j, k)] = vx;
    if (j == 0) by[face_store(g, 1, i, g.n[1], k)] = vy;
    if (k == 0) bz[face_store(g, 2, i, j, g.n[2])] = vz;
}

__global__ void k_curl_potential_adjoint(Geom g, const double *lbx, const double *lby,
                                         const double *lbz, double *lax, double *lay, double *laz)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    int x[3];
    cell_coords(g, t, x);
    const int i = x[0], j = x[1], k = x[2];
    // cotangent of face (d; a, b, c) with the duplicate plane's folded onto plane 0
    auto lb = [&](int d, const double *p, int a, int b2, int c2) {
        const int q[3] = {wrapc(a, g.n[0]), wrapc(b2, g.n[1]), wrapc(c2, g.n[2])};
        double v = p[face_store(g, d, q[0], q[1], q[2])];
        if (q[d] == 0) {
            int r[3] = {q[0], q[1], q[2]};
            r[d] = g.n[d];
            v += p[face_store(g, d, r[0], r[1], r[2])];
        }
        return v;
    };
    lax[t] = (lb(1, lby, i, j, k - 1) - lb(1, lby, i, j, k)) / g.dl[2]
             + (lb(2, lbz, i, j, k) - lb(2, lbz, i, j - 1, k)) / g.dl[1];
    lay[t] = (lb(0, lbx, i, j, k) - lb(0, lbx, i, j, k - 1)) / g.dl[2]
             + (lb(2, lbz, i - 1, j, k) - lb(2, lbz, i, j, k)) / g.dl[0];
    laz[t] = (lb(0, lbx, i, j - 1, k) - lb(0, lbx, i, j, k)) / g.dl[1]
             + (lb(1, lby, i, j, k) - lb(1, lby, i - 1, j, k)) / g.dl[0];
}

}  // namespace vlct

using namespace vlct;

extern "C" {

static bool periodic_grid(const vlct_grid *g)
{
    return grid_ok(g) && g->bc[0] == VLCT_BC_PERIODIC && g->bc[1] == VLCT_BC_PERIODIC &&
           g->bc[2] == VLCT_BC_PERIODIC;
}

int vlct_curl_potential(const vlct_grid *vg, const double *ax, const double *ay, const double *az,
                        double *bx, double *by, double *bz, void *stream)
{
    if (!grid_ok(vg) || !ax || !ay || !az || !bx || !by || !bz) return VLCT_EINVAL;
    if (!periodic_grid(vg)) return VLCT_EUNSUPPORTED;
    const Geom g = make_geom(vg);
    const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    k_curl_potential<<<nblocks(N), kBlock, 0, static_cast<hipStream_t>(stream)>>>(g, ax, ay, az,
                                                                                 bx, by, bz);
    return hipGetLastError() == hipSuccess ? VLCT_OK : VLCT_EHIP;
}

int vlct_curl_potential_adjoint(const vlct_grid *vg, const double *lbx, const double *lby,
                                const double *lbz, double *lax, double *lay, double *laz,
                                void *stream)
{
    if (!grid_ok(vg) || !lbx || !lby || !lbz || !lax || !lay || !laz) return VLCT_EINVAL;
    if (!periodic_grid(vg)) return VLCT_EUNSUPPORTED;
    const Geom g = make_geom(vg);
    const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    k_curl_potential_adjoint<<<nblocks(N), kBlock, 0, static_cast<hipStream_t>(stream)>>>(
        g, lbx, lby, lbz, lax, lay, laz);
    return hipGetLastError() == hipSuccess ? VLCT_OK : VLCT_EHIP;
}

size_t vlct_adjoint_workspace_bytes(const vlct_grid *g)
{
    if (!grid_ok(g)) return 0;
    return ad_layout(make_geom(g), false).total;
}

size_t vlct_adjoint_taped_workspace_bytes(const vlct_grid *g)
{
    if (!grid_ok(g)) return 0;
    return ad_layout(make_geom(g), true).total;
}

int vlct_step_adjoint(const vlct_grid *vg, const vlct_state *in, const vlct_state *lam_out,
                      const vlct_state *lam_in, const double *dt_dev, void *ws, size_t ws_bytes,
                      void *stream)
{
    int rc = adjoint_args(vg, in, lam_out, lam_in, dt_dev);
    if (rc) return rc;
    const Geom g = make_geom(vg);
    const AdLayout L = ad_layout(g, false);
    if (!ws || ws_bytes < L.total) return VLCT_EWORKSPACE;
    char *b = static_cast<char *>(ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto arr = [&](size_t off) { return reinterpret_cast<double *>(b + off); };
    Prims P[2];
    for (int h = 0; h < 2; ++h)
        for (int f = 0; f < 8; ++f) P[h].w[f] = arr(L.prims[h] + f * align_up(L.prims_len * 8));
    StateW half;
    for (int f = 0; f < 8; ++f) {
        if (f < 5) half.u[f] = arr(L.half[f]); else half.b[f - 5] = arr(L.half[f]);
    }
    Flux F[2];
    uint8_t *side[2][3];
    Sides sides[2];
    for (int h = 0; h < 2; ++h) {
        F[h] = bind_flux(b, L.flux[h], L.flux_len);
        for (int d = 0; d < 3; ++d) {
            side[h][d] = reinterpret_cast<uint8_t *>(b + L.side[h][d]);
            sides[h].s[d] = side[h][d];
        }
    }
    // forward intermediates at U^n (the kernels of vlct_step)
    const StateP sin = as_const(in);
    rc = launch_prims(g, sin, P[0], nullptr, s);
    if (!rc) rc = launch_fluxes(g, sin, P[0], F[0], VLCT_RECON_PCM, nullptr, s);
    if (!rc) rc = launch_pack_sides(g, F[0], side[0], s);
    if (!rc) rc = launch_ct(g, false, P[0], F[0], sin, half, dt_dev, nullptr, s);
    const StateP hc = as_const(half);
    if (!rc) rc = launch_prims(g, hc, P[1], nullptr, s);
    if (!rc) rc = launch_fluxes(g, hc, P[1], F[1], vg->recon, nullptr, s);
    if (!rc) rc = launch_pack_sides(g, F[1], side[1], s);
    if (rc) return rc;
    return adjoint_core(vg, g, L, b, sin, hc, sides, true, lam_out, lam_in, dt_dev, s);
}

int vlct_step_adjoint_taped(const vlct_grid *vg, const vlct_state *in, const vlct_state *lam_out,
                            const vlct_state *lam_in, const double *dt_dev, const void *tape,
                            size_t tape_bytes, void *ws, size_t ws_bytes, void *stream)
{
    int rc = adjoint_args(vg, in, lam_out, lam_in, dt_dev);
    if (rc) return rc;
    const Geom g = make_geom(vg);
    const AdLayout L = ad_layout(g, true);
    const TapeLayout T = tape_layout(g.n);
    if (!ws || ws_bytes < L.total || !tape || tape_bytes < T.total) return VLCT_EWORKSPACE;
    const char *tb = static_cast<const char *>(tape);
    StateP hc;
    for (int f = 0; f < 8; ++f) {
        const double *a = reinterpret_cast<const double *>(tb + T.half[f]);
        if (f < 5) hc.u[f] = a; else hc.b[f - 5] = a;
    }
    Sides sides[2];
    for (int h = 0; h < 2; ++h)
        for (int d = 0; d < 3; ++d) sides[h].s[d] = reinterpret_cast<const uint8_t *>(tb + T.side[h][d]);
    return adjoint_core(vg, g, L, static_cast<char *>(ws), as_const(in), hc, sides, false,
                        lam_out, lam_in, dt_dev, static_cast<hipStream_t>(stream));
}

}  // extern "C"
