// vlct.hip -- one VL+CT step of 3D ideal MHD on gfx950 (Caddy & Schneider,
// "Cholla-MHD", Sec. 2.2) behind the C ABI of include/vlct.h.
//
// Step structure (all kernels on the caller's stream, state resident in HBM):
//   stage(U^n, PCM)        : prims -> 3 x (HLLD fluxes) -> CT edge EMFs + half update
//   stage(U^{n+1/2}, PLMC) : prims -> 3 x (reconstruction + HLLD)
//                            -> CT edge EMFs + full update from U^n, with the
//                               per-block CFL maxima of the new state -> final
//                               next-dt reduction (an in-place step reduces the
//                               CFL condition in a kernel of its own)
// Boundary conditions enter only through the primitive kernel, which fills a
// ghost-padded primitive array by index mapping (wrap / clamp), and through
// face-index mapping when the stored normal field is read.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "vlct_common.hpp"
#include "mhd_physics.hpp"

namespace vlct {

// ---------------------------------------------------------------------------
// logical block counts of the kernels (host launches and batch offsets)
// ---------------------------------------------------------------------------
constexpr int kRowFaces = kBlock - 1;
constexpr int kMarch = 16;
constexpr int kTx = 64, kTy = 8;  // CT column tile (z planes per block: Geom::ct_planes)
constexpr int kCt = kTx * kTy;  // threads of a CT block: one per column of the tile

// tile variants a batched step can give each instance (its plan byte: CT
// variant in the low nibble, march variant in the high nibble); variant 0 is
// the single-instance CT tile and the 16-face march (single steps on small
// grids march 8 faces; every variant computes the same bits)
constexpr int kCtVariants = 3;     // CT column tiles 64 x 8, 32 x 16, 16 x 32 (kCt threads)
constexpr int kMarchVariants = 3;  // march segments of 16, 32 and 8 faces
__host__ __device__ constexpr int ct_tx(int v) { return v == 0 ? 64 : (v == 1 ? 32 : 16); }
__host__ __device__ constexpr int ct_ty(int v) { return kCt / ct_tx(v); }
__host__ __device__ constexpr int march_len(int v) { return v == 0 ? 16 : (v == 1 ? 32 : 8); }

__host__ __device__ __forceinline__ idx_t nblk_prims(const Geom &g)
{
    return ((idx_t)g.p[0] * g.p[1] * g.p[2] + kBlock - 1) / kBlock;
}
__host__ __device__ __forceinline__ idx_t flux_dim3(const Geom &g, int d)
{
    return flux_dim(g.n, d, 0) * flux_dim(g.n, d, 1) * flux_dim(g.n, d, 2);
}
__host__ __device__ __forceinline__ idx_t nblk_flux(const Geom &g, int d)
{
    return (flux_dim3(g, d) + kBlock - 1) / kBlock;
}
__host__ __device__ __forceinline__ idx_t nblk_row(const Geom &g)
{
    const idx_t items = (idx_t)(g.n[0] + 2) * (g.n[1] + 2) * (g.n[2] + 2);
    return (items - 1 + kRowFaces - 1) / kRowFaces;
}
__host__ __device__ __forceinline__ idx_t nblk_march(const Geom &g, int d, int m = kMarch)
{
    const int t = d == 1 ? 2 : 1;
    const idx_t cols = (idx_t)(g.n[0] + 2) * (g.n[t] + 2);
    return ((cols + kBlock - 1) / kBlock) * ((g.n[d] + 1 + m - 1) / m);
}
__host__ __device__ __forceinline__ idx_t nblk_ct(const Geom &g, int tx = kTx, int ty = kTy)
{
    const int ntx = (g.n[0] + (g.bc[0] == VLCT_BC_OUTFLOW) + tx - 1) / tx;
    const int nty = (g.n[1] + (g.bc[1] == VLCT_BC_OUTFLOW) + ty - 1) / ty;
    const int ntz = (g.n[2] + g.ct_planes - 1) / g.ct_planes;
    return (idx_t)ntx * nty * ntz;
}
__host__ __device__ __forceinline__ idx_t nblk_dt(const Geom &g)
{
    return ((idx_t)g.n[0] * g.n[1] * g.n[2] + kBlock - 1) / kBlock;
}

// ---------------------------------------------------------------------------
// primitive variables on the ghost-padded grid (Sec. 2.1; B_cc = face average,
// Step 1); the boundary conditions are applied here by index mapping
// ---------------------------------------------------------------------------
// primitives of one cell from its conserved variables u and cell-centred
// field, floored (the conserved state is never changed), stored at padded
// index o; returns the floor status bits
__device__ __forceinline__ uint32_t prims_store(const Geom &g, const Prims &P, idx_t o,
                                                const double u[5], double bcx, double bcy,
                                                double bcz)
{
    double d = u[0];
    uint32_t st = 0;
    if (!(d >= kFloorRho)) { d = kFloorRho; st |= kStatusDensityFloor; }
    const double id = 1.0 / d;
    const double vx = u[1] * id, vy = u[2] * id, vz = u[3] * id;
    const double ke = 0.5 * d * (vx * vx + vy * vy + vz * vz);
    const double me = 0.5 * (bcx * bcx + bcy * bcy + bcz * bcz);
    double pr = (g.gamma - 1.0) * (u[4] - ke - me);
    if (!(pr >= kFloorP)) { pr = kFloorP; st |= kStatusPressureFloor; }
    P.w[0][o] = d;
    P.w[1][o] = vx;
    P.w[2][o] = vy;
    P.w[3][o] = vz;
    P.w[4][o] = pr;
    P.w[5][o] = bcx;
    P.w[6][o] = bcy;
    P.w[7][o] = bcz;
    return st;
}

// primitives of padded cell (i, j, k), i, j, k in [-G, n + G - 1], with the
// boundary conditions applied by index mapping
__device__ __forceinline__ uint32_t prims_cell(const Geom &g, const StateP &s, const Prims &P,
                                               int i, int j, int k)
{
    const int mi = map_cell(i, g.n[0], g.bc[0]);
    const int mj = map_cell(j, g.n[1], g.bc[1]);
    const int mk = map_cell(k, g.n[2], g.bc[2]);
    const idx_t c = cell_store(g, mi, mj, mk);
    const double bx0 = s.b[0][face_store(g, 0, map_face(i, g.n[0], g.bc[0]), mj, mk)];
    const double bx1 = s.b[0][face_store(g, 0, map_face(i + 1, g.n[0], g.bc[0]), mj, mk)];
    const double by0 = s.b[1][face_store(g, 1, mi, map_face(j, g.n[1], g.bc[1]), mk)];
    const double by1 = s.b[1][face_store(g, 1, mi, map_face(j + 1, g.n[1], g.bc[1]), mk)];
    const double bz0 = s.b[2][face_store(g, 2, mi, mj, map_face(k, g.n[2], g.bc[2]))];
    const double bz1 = s.b[2][face_store(g, 2, mi, mj, map_face(k + 1, g.n[2], g.bc[2]))];
    const double u[5] = {s.u[0][c], s.u[1][c], s.u[2][c], s.u[3][c], s.u[4][c]};
    return prims_store(g, P, pidx(g, i, j, k), u, 0.5 * (bx0 + bx1), 0.5 * (by0 + by1),
                       0.5 * (bz0 + bz1));
}

__device__ __forceinline__ void prims_body(const Geom &g, const StateP &s, const Prims &P,
                                           uint32_t *status, idx_t b)
{
    const idx_t tot = (idx_t)g.p[0] * g.p[1] * g.p[2];
    const idx_t t = b * kBlock + threadIdx.x;
    if (t >= tot) return;
    const int pi = (int)(t % g.p[0]);
    const idx_t r = t / g.p[0];
    const int pj = (int)(r % g.p[1]);
    const int pk = (int)(r / g.p[1]);
    const uint32_t st = prims_cell(g, s, P, pi - kGhost, pj - kGhost, pk - kGhost);
    if (st && status) atomicOr(status, st);
}

// ghost layers only: the padded cells outside the grid, enumerated as the
// z-ghost planes, then the y-ghost rows of interior planes, then the x-ghost
// cells of interior rows
__host__ __device__ __forceinline__ idx_t ghost_cells(const Geom &g)
{
    return (idx_t)g.p[0] * g.p[1] * g.p[2] - (idx_t)g.n[0] * g.n[1] * g.n[2];
}

__device__ __forceinline__ void prims_ghost_body(const Geom &g, const StateP &s, const Prims &P,
                                                 uint32_t *status, idx_t b)
{
    const idx_t t = b * kBlock + threadIdx.x;
    if (t >= ghost_cells(g)) return;
    const int px = g.p[0], py = g.p[1], G2 = 2 * kGhost;
    const idx_t n1 = (idx_t)G2 * px * py, n2 = (idx_t)g.n[2] * G2 * px;
    int i, j, k;
    if (t < n1) {
        const int q = (int)(t / ((idx_t)px * py));
        const idx_t r = t % ((idx_t)px * py);
        k = q < kGhost ? q - kGhost : g.n[2] + q - kGhost;
        j = (int)(r / px) - kGhost;
        i = (int)(r % px) - kGhost;
    } else if (t < n1 + n2) {
        const idx_t r = t - n1;
        k = (int)(r / ((idx_t)G2 * px));
        const int q = (int)((r / px) % G2);
        j = q < kGhost ? q - kGhost : g.n[1] + q - kGhost;
        i = (int)(r % px) - kGhost;
    } else {
        const idx_t r = t - n1 - n2;
        k = (int)(r / ((idx_t)g.n[1] * G2));
        j = (int)((r / G2) % g.n[1]);
        const int q = (int)(r % G2);
        i = q < kGhost ? q - kGhost : g.n[0] + q - kGhost;
    }
    const uint32_t st = prims_cell(g, s, P, i, j, k);
    if (st && status) atomicOr(status, st);
}

// sweep-frame state of a padded cell for axis D
template <int D>
__device__ __forceinline__ W7 load_w7(const Prims &P, idx_t o)
{
    constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
    return W7{P.w[0][o], P.w[1 + D][o], P.w[1 + t1][o], P.w[1 + t2][o],
              P.w[4][o], P.w[5 + t1][o], P.w[5 + t2][o]};
}

// ---------------------------------------------------------------------------
// PCM interface states + HLLD on every face of axis D (Steps 2-3)
// ---------------------------------------------------------------------------
template <int D, int RECON>
__device__ __forceinline__ void flux_pcm_body(const Geom &g, const StateP &s, const Prims &P,
                                              const Flux &F, uint32_t *status, idx_t b)
{
    const idx_t X = flux_dim(g.n, D, 0), Y = flux_dim(g.n, D, 1), Z = flux_dim(g.n, D, 2);
    const idx_t t = b * kBlock + threadIdx.x;
    if (t >= X * Y * Z) return;
    int x[3];
    x[0] = (int)(t % X) - (D != 0);
    const idx_t r = t / X;
    x[1] = (int)(r % Y) - (D != 1);
    x[2] = (int)(r / Y) - (D != 2);
    // cells along D around the face x[D] - 1/2
    auto cell_at = [&](int off) {
        int c[3] = {x[0], x[1], x[2]};
        c[D] += off;
        return pidx(g, c[0], c[1], c[2]);
    };
    static_assert(RECON == VLCT_RECON_PCM, "k_flux serves the PCM predictor");
    const W7 wl = load_w7<D>(P, cell_at(-1));
    const W7 wr = load_w7<D>(P, cell_at(0));
    const uint32_t st = 0;
    // stored normal field of this face (transverse indices mapped like cells)
    int m[3];
#pragma unroll
    for (int e = 0; e < 3; ++e)
        m[e] = e == D ? map_face(x[e], g.n[e], g.bc[e]) : map_cell(x[e], g.n[e], g.bc[e]);
    const double bn = s.b[D][face_store(g, D, m[0], m[1], m[2])];
    double f[7], upw;
    hlld(wl, wr, bn, g.gamma, g.gm1i, f, upw);
    if (st && status) atomicOr(status, st);
#pragma unroll
    for (int c = 0; c < 7; ++c) F.f[D][c][t] = f[c];
    F.sg[D][t] = (int8_t)upw;
}

// ---------------------------------------------------------------------------
// corrector fluxes without duplicated reconstruction: every cell is
// reconstructed once per axis and its two interface states feed the faces on
// either side.
//
// x axis: a block of 256 threads reconstructs 256 consecutive cells of one
// row; the high-face states go through LDS to the right neighbour, which
// solves the Riemann problem of the face between them (255 faces per block).
// ---------------------------------------------------------------------------
template <int RECON>
__device__ __forceinline__ void recon_cell(const Prims &P, const Geom &g, int D, const int c[3],
                                           W7 &fm, W7 &fp)
{
    (void)g;
    auto at = [&](int off) {
        int q[3] = {c[0], c[1], c[2]};
        q[D] += off;
        return pidx(g, q[0], q[1], q[2]);
    };
    const idx_t c0 = at(0);
    const double bn = P.w[5 + D][c0];
    constexpr bool kChar = RECON == VLCT_RECON_PLMC || RECON == VLCT_RECON_PPMC;
    constexpr bool kLinear = RECON == VLCT_RECON_PLMC || RECON == VLCT_RECON_PLMP;
    if (D == 0) {
        if (kLinear)
            plmc<kChar>(load_w7<0>(P, at(-1)), load_w7<0>(P, c0), load_w7<0>(P, at(1)), bn,
                        g.gamma, fm, fp);
        else
            ppmc<kChar>(load_w7<0>(P, at(-2)), load_w7<0>(P, at(-1)), load_w7<0>(P, c0),
                        load_w7<0>(P, at(1)), load_w7<0>(P, at(2)), bn, g.gamma, fm, fp);
    }
}

template <int RECON>
__device__ __forceinline__ void recon_x_body(const Geom &g, const StateP &s, const Prims &P,
                                             const Flux &F, uint32_t *status, idx_t b)
{
    // items = (row, cell) with cells -1..nx of every row (j in [-1, ny],
    // k in [-1, nz]) in one flat sequence; a block reconstructs 256
    // consecutive items and solves the face between each item and its left
    // neighbour in the same row; consecutive blocks overlap by one item
    __shared__ double lds[7][kBlock];
    const int nx = g.n[0];
    const idx_t per_row = nx + 2;
    const idx_t items = per_row * (idx_t)(g.n[1] + 2) * (g.n[2] + 2);
    const idx_t nblk = (items - 1 + kRowFaces - 1) / kRowFaces;
    const int t = threadIdx.x;
    const idx_t q = b * kRowFaces + t;
    const bool have = b < nblk && q < items;
    const idx_t row = q / per_row;
    const int c = (int)(q - row * per_row) - 1;
    const int Y = g.n[1] + 2;
    const int j = (int)(row % Y) - 1;
    const int k = (int)(row / Y) - 1;
    W7 fm{}, fp{};
    uint32_t st = 0;
    if (have) {
        const int cc[3] = {c, j, k};
        recon_cell<RECON>(P, g, 0, cc, fm, fp);
        st |= floor_state(fm);
        st |= floor_state(fp);
    }
    lds[0][t] = fp.d; lds[1][t] = fp.u; lds[2][t] = fp.v; lds[3][t] = fp.w;
    lds[4][t] = fp.p; lds[5][t] = fp.by; lds[6][t] = fp.bz;
    __syncthreads();
    if (t >= 1 && have && c >= 0) {
        const W7 wl{lds[0][t - 1], lds[1][t - 1], lds[2][t - 1], lds[3][t - 1],
                    lds[4][t - 1], lds[5][t - 1], lds[6][t - 1]};
        const int mj = map_cell(j, g.n[1], g.bc[1]), mk = map_cell(k, g.n[2], g.bc[2]);
        const double bn = s.b[0][face_store(g, 0, map_face(c, nx, g.bc[0]), mj, mk)];
        double f[7], upw;
        hlld(wl, fm, bn, g.gamma, g.gm1i, f, upw);
        const idx_t o = fidx(g, 0, c, j, k);
#pragma unroll
        for (int v = 0; v < 7; ++v) F.f[0][v][o] = f[v];
        F.sg[0][o] = (int8_t)upw;
    }
    if (st && status) atomicOr(status, st);
}

// y and z axes: one thread per transverse column (columns flattened with x
// fastest, so loads and stores are coalesced); each thread marches along the
// axis through a segment of M faces, keeping the stencil and the previous
// cell's high-face state in registers (one extra reconstruction per segment).
template <int D, int RECON, int M = kMarch>
__device__ __forceinline__ void march_body(const Geom &g, const StateP &s, const Prims &P,
                                           const Flux &F, uint32_t *status, idx_t b)
{
    constexpr int T = D == 1 ? 2 : 1;         // the transverse axis other than x
    constexpr bool kChar = RECON == VLCT_RECON_PLMC || RECON == VLCT_RECON_PPMC;
    constexpr int R = (RECON == VLCT_RECON_PLMC || RECON == VLCT_RECON_PLMP) ? 1 : 2;
    const int nD = g.n[D];
    // columns (i, it), i in [-1, nx], it in [-1, n_T], flattened with i fastest
    const idx_t cols = (idx_t)(g.n[0] + 2) * (g.n[T] + 2);
    const idx_t ncb = (cols + kBlock - 1) / kBlock;
    const int nseg = (nD + 1 + M - 1) / M;
    const int seg = (int)(b / ncb);
    const idx_t col = (b % ncb) * kBlock + threadIdx.x;
    if (seg >= nseg || col >= cols) return;
    const int i = (int)(col % (g.n[0] + 2)) - 1;
    const int it = (int)(col / (g.n[0] + 2)) - 1;
    const int s0 = seg * M;
    const int s1 = min(s0 + M, nD + 1);  // faces [s0, s1)
    int x[3];
    x[0] = i;
    x[T] = it;
    auto pid = [&](int along) {
        int q[3] = {x[0], x[1], x[2]};
        q[D] = along;
        return pidx(g, q[0], q[1], q[2]);
    };
    // stencil window of cells c-R .. c+R for c = s0 - 1
    W7 win[2 * R + 1];
    double bnc[2 * R + 1];
#pragma unroll
    for (int q = 0; q < 2 * R + 1; ++q) {
        const idx_t o = pid(s0 - 1 - R + q);
        win[q] = load_w7<D>(P, o);
        bnc[q] = P.w[5 + D][o];
    }
    uint32_t st = 0;
    W7 prev{};
    const int mt = map_cell(it, g.n[T], g.bc[T]);
    const int mi = map_cell(i, g.n[0], g.bc[0]);
    for (int c = s0 - 1; c < s1; ++c) {
        W7 fm, fp;
        if constexpr (R == 1)
            plmc<kChar>(win[0], win[1], win[2], bnc[1], g.gamma, fm, fp);
        else
            ppmc<kChar>(win[0], win[1], win[2], win[3], win[4], bnc[2], g.gamma, fm, fp);
        st |= floor_state(fm);
        st |= floor_state(fp);
        if (c >= s0) {
            int m[3];
            m[0] = mi;
            m[T] = mt;
            m[D] = map_face(c, nD, g.bc[D]);
            const double bn = s.b[D][face_store(g, D, m[0], m[1], m[2])];
            double f[7], upw;
            hlld(prev, fm, bn, g.gamma, g.gm1i, f, upw);
            int q[3] = {x[0], x[1], x[2]};
            q[D] = c;
            const idx_t o = fidx(g, D, q[0], q[1], q[2]);
#pragma unroll
            for (int v = 0; v < 7; ++v) F.f[D][v][o] = f[v];
            F.sg[D][o] = (int8_t)upw;
        }
        prev = fp;
        if (c + 1 < s1) {
#pragma unroll
            for (int q = 0; q < 2 * R; ++q) {
                win[q] = win[q + 1];
                bnc[q] = bnc[q + 1];
            }
            const idx_t o = pid(c + 1 + R);
            win[2 * R] = load_w7<D>(P, o);
            bnc[2 * R] = P.w[5 + D][o];
        }
    }
    if (st && status) atomicOr(status, st);
}

// ---------------------------------------------------------------------------
// CFL condition of one cell (Step 1, Eq. dt): max_l (|v_l| + c_f,l) / d_l from
// its conserved variables and cell-centred field (face averages); floored
// rho / P as in the primitive recovery, the floors reported in `st`
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cell_cfl(const Geom &g, double d, double mx, double my,
                                           double mz, double e, const double b[3], uint32_t &st)
{
    if (!(d >= kFloorRho)) { d = kFloorRho; st |= kStatusDensityFloor; }
    const double id = 1.0 / d;
    const double v[3] = {mx * id, my * id, mz * id};
    const double ke = 0.5 * d * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double me = 0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    double p = (g.gamma - 1.0) * (e - ke - me);
    if (!(p >= kFloorP)) { p = kFloorP; st |= kStatusPressureFloor; }
    double m = 0.0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const double cf = fast_speed(d, p, b[l], b[(l + 1) % 3], b[(l + 2) % 3], g.gamma);
        m = fmax(m, (fabs(v[l]) + cf) / g.dl[l]);
    }
    return m;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// ---------------------------------------------------------------------------
// CT edge EMFs (Step 4 / Step 8; Eqs. emf-edge, emf-upwind-slope, emf-slope)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double upwind(double s, double lo, double hi)
{
    return s > 0.0 ? lo : (s < 0.0 ? hi : 0.5 * (lo + hi));
}

// the edge field from the EMFs and upwind indicators of its four faces and the
// reference fields of its four cells: B-faces at x0 and x0 - e_C, C-faces at
// x0 and x0 - e_B
__device__ __forceinline__ double edge_combine(double eb_c, double eb_cm, double ec_b,
                                               double ec_bm, double sb_c, double sb_cm,
                                               double sc_b, double sc_bm, double r00, double r10,
                                               double r01, double r11)
{
    const double avg = 0.25 * (eb_c + eb_cm + ec_b + ec_bm);
    const double t1 = upwind(sb_c, ec_bm - r10, ec_b - r00);
    const double t2 = upwind(sb_cm, ec_bm - r11, ec_b - r01);
    const double t3 = upwind(sc_b, eb_cm - r01, eb_c - r00);
    const double t4 = upwind(sc_bm, eb_cm - r11, eb_c - r10);
    return avg + 0.25 * (t1 + t2 + t3 + t4);
}

template <int A>
__device__ __forceinline__ double edge_emf(const Geom &g, const Flux &F, int i, int j, int k,
                                           double r00, double r10, double r01, double r11)
{
    // r00, r10, r01, r11: cell-centred -(v x B)_A of the cells at x0, x0 - e_B,
    // x0 - e_C and x0 - e_B - e_C around the edge
    constexpr int B = (A + 1) % 3, C = (A + 2) % 3;
    int x0[3] = {i, j, k};
    int xb[3] = {i, j, k};
    xb[B] -= 1;
    int xc[3] = {i, j, k};
    xc[C] -= 1;
    const idx_t fb_c = fidx(g, B, x0[0], x0[1], x0[2]);
    const idx_t fb_cm = fidx(g, B, xc[0], xc[1], xc[2]);
    const idx_t fc_b = fidx(g, C, x0[0], x0[1], x0[2]);
    const idx_t fc_bm = fidx(g, C, xb[0], xb[1], xb[2]);
    // B-face EMF component A = -F_B[B_t1]; C-face EMF component A = +F_C[B_t2]
    return edge_combine(-F.f[B][5][fb_c], -F.f[B][5][fb_cm], F.f[C][6][fc_b], F.f[C][6][fc_bm],
                        F.sg[B][fb_c], F.sg[B][fb_cm], F.sg[C][fc_b], F.sg[C][fc_bm], r00, r10,
                        r01, r11);
}

// E_x (A = 0) or E_y (A = 1) at the half plane k - 1/2 for a block marching up
// in z: of its four faces, the one at x0 - e_z (the B-face for E_x, the
// C-face for E_y) is the face at x0 of the half plane below, so its EMF and
// upwind indicator come in through (ez, sz) and those at x0 go out through
// them for the next half plane.  FIRST: the lower face is read, as edge_emf
// reads it.
template <int A, bool FIRST>
__device__ __forceinline__ double edge_emf_zcarry(const Geom &g, const Flux &F, int i, int j,
                                                  int k, double r00, double r10, double r01,
                                                  double r11, double &ez, int8_t &sz)
{
    static_assert(A == 0 || A == 1, "the z-marching carry serves E_x and E_y");
    constexpr int B = (A + 1) % 3, C = (A + 2) % 3;
    constexpr int Z = A == 0 ? B : C;  // the face axis whose faces stack along z
    constexpr int T = A == 0 ? C : B;  // the face axis whose two faces share the plane
    const idx_t fz_hi = fidx(g, Z, i, j, k);
    int xt[3] = {i, j, k};
    xt[A == 0 ? B : C] -= 1;  // the in-plane neighbour of the T-faces
    const idx_t ft_0 = fidx(g, T, i, j, k), ft_1 = fidx(g, T, xt[0], xt[1], xt[2]);
    // EMF component A: -F_B[B_t1] on a B-face, +F_C[B_t2] on a C-face
    constexpr int zcomp = Z == B ? 5 : 6, tcomp = T == B ? 5 : 6;
    double e_lo, s_lo;
    if (FIRST) {
        const idx_t fz_lo = fidx(g, Z, i, j, k - 1);
        e_lo = Z == B ? -F.f[Z][zcomp][fz_lo] : F.f[Z][zcomp][fz_lo];
        s_lo = F.sg[Z][fz_lo];
    } else {
        e_lo = ez;
        s_lo = sz;
    }
    const double e_hi = Z == B ? -F.f[Z][zcomp][fz_hi] : F.f[Z][zcomp][fz_hi];
    const int8_t s_hi = F.sg[Z][fz_hi];
    const double et0 = T == B ? -F.f[T][tcomp][ft_0] : F.f[T][tcomp][ft_0];
    const double et1 = T == B ? -F.f[T][tcomp][ft_1] : F.f[T][tcomp][ft_1];
    const double st0 = F.sg[T][ft_0], st1 = F.sg[T][ft_1];
    ez = e_hi;
    sz = s_hi;
    if (A == 0)  // B = y stacked along z (x0 - e_C = lower), C = z faces at x0 and x0 - e_y
        return edge_combine(e_hi, e_lo, et0, et1, (double)s_hi, s_lo, st0, st1, r00, r10, r01,
                            r11);
    else  // B = z faces at x0 and x0 - e_x, C = x stacked along z (x0 - e_B = lower)
        return edge_combine(et0, et1, e_hi, e_lo, st0, st1, (double)s_hi, s_lo, r00, r10, r01,
                            r11);
}

// ---------------------------------------------------------------------------
// fused CT + update (Steps 4-5 and 8-9): a block owns a 64 x 8 column tile and
// marches along z.  For each plane k it computes the edge fields it needs once
// into LDS -- E_z of plane k, E_x / E_y of the plane above (k+1/2); those of
// the plane below are kept from the previous iteration -- and then updates the
// plane's cells and the faces owned by them.  Same arithmetic as k_edges and
// k_update, without the round trip of the edge arrays through HBM.
// ---------------------------------------------------------------------------

// DT (full step only): the CFL condition of the updated cells is reduced on
// the way, one maximum per block into partial[b]; the cell-centred field
// takes the cell's high faces recomputed from the same edge fields as the
// threads (or blocks) that own them.
template <bool FULL, int TX = kTx, int TY = kTy, bool DT = false>
__device__ __forceinline__ void ct_body(const Geom &g, const Prims &P, const Flux &F,
                                        const StateP &base, const StateW &out,
                                        const double *dt_dev, uint32_t *status, idx_t b,
                                        double *partial = nullptr)
{
    static_assert(FULL || !DT, "the CFL reduction belongs to the full step");
    __shared__ double sez[TY + 1][TX + 1];
    __shared__ double sex[2][TY + 1][TX];
    __shared__ double sey[2][TY][TX + 1];
    // cell-centred -(v x B) of the tile plus a one-cell halo below in x and y,
    // two planes in flight: plane kk lives in slot (kk - k0 + 1) & 1
    __shared__ double sref[2][3][TY + 2][TX + 2];
    // EMF and upwind indicator of each horizontal edge's face stacked along z
    __shared__ double szc_e[(TY + 1) * TX + TY * (TX + 1)];
    __shared__ int8_t szc_s[(TY + 1) * TX + TY * (TX + 1)];
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    // positions owned by threads: cells/faces i in [0, ex), j in [0, ey)
    const int ex = nx + (g.bc[0] == VLCT_BC_OUTFLOW), ey = ny + (g.bc[1] == VLCT_BC_OUTFLOW);
    const int tz = g.ct_planes;
    const int ntx = (ex + TX - 1) / TX, nty = (ey + TY - 1) / TY, ntz = (nz + tz - 1) / tz;
    if (b >= (idx_t)ntx * nty * ntz) return;
    const int bx = (int)(b % ntx), by = (int)((b / ntx) % nty), bz = (int)(b / ((idx_t)ntx * nty));
    const int i0 = bx * TX, j0 = by * TY, k0 = bz * tz, k1 = min(k0 + tz, nz);
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int i = i0 + tx, j = j0 + ty;
    const double dt = FULL ? dt_dev[0] : 0.5 * dt_dev[0];
    const double cx = dt / g.dl[0], cy = dt / g.dl[1], cz = dt / g.dl[2];
    constexpr int NEZ = (TY + 1) * (TX + 1), NEX = (TY + 1) * TX, NEY = TY * (TX + 1);

    constexpr int NREF = (TY + 2) * (TX + 2);
    auto slot = [&](int kk) { return (kk - k0 + 1) & 1; };
    // reference EMFs of plane kk (cells up to n: the highest edges are at n - 1/2)
    auto stage_ref = [&](int kk) {
        const int sl = slot(kk);
        for (int q = threadIdx.x; q < NREF; q += (TX * TY)) {
            const int a = q % (TX + 2), c = q / (TX + 2), ii = i0 - 1 + a, jj = j0 - 1 + c;
            if (ii <= nx && jj <= ny) {
                const idx_t o = pidx(g, ii, jj, kk);
                const double vx = P.w[1][o], vy = P.w[2][o], vz = P.w[3][o];
                const double bx = P.w[5][o], by = P.w[6][o], bz = P.w[7][o];
                sref[sl][0][c][a] = -(vy * bz - vz * by);
                sref[sl][1][c][a] = -(vz * bx - vx * bz);
                sref[sl][2][c][a] = -(vx * by - vy * bx);
            }
        }
    };
    // LDS coordinates of cell (ii, jj): [jj - j0 + 1][ii - i0 + 1]
    // edge q of the plane kk - 1/2 (E_x for q < NEX, else E_y, at edge index
    // kk) into slot h; szc_e / szc_s[q] carry the EMF and upwind indicator of
    // its face stacked along z from one half plane to the next (first: read
    // them).  Only the thread working on edge q touches entry q within a plane.
    auto horizontal_edge = [&](int q, int kk, int h, bool first) {
        const int up = slot(kk), dn = slot(kk - 1);
        const int qe = q;
        if (q < NEX) {
            const int a = q % TX, c = q / TX, ii = i0 + a, jj = j0 + c;
            // E_x at (ii, jj - 1/2, kk - 1/2): B = y, C = z
            if (ii < nx && jj <= ny) {
                const double r00 = sref[up][0][c + 1][a + 1], r10 = sref[up][0][c][a + 1];
                const double r01 = sref[dn][0][c + 1][a + 1], r11 = sref[dn][0][c][a + 1];
                sex[h][c][a] = first ? edge_emf_zcarry<0, true>(g, F, ii, jj, kk, r00, r10, r01, r11,
                                                                szc_e[qe], szc_s[qe])
                                     : edge_emf_zcarry<0, false>(g, F, ii, jj, kk, r00, r10, r01, r11,
                                                                 szc_e[qe], szc_s[qe]);
            }
        } else {
            q -= NEX;
            const int a = q % (TX + 1), c = q / (TX + 1), ii = i0 + a, jj = j0 + c;
            // E_y at (ii - 1/2, jj, kk - 1/2): B = z, C = x
            if (ii <= nx && jj < ny) {
                const double r00 = sref[up][1][c + 1][a + 1], r10 = sref[dn][1][c + 1][a + 1];
                const double r01 = sref[up][1][c + 1][a], r11 = sref[dn][1][c + 1][a];
                sey[h][c][a] = first ? edge_emf_zcarry<1, true>(g, F, ii, jj, kk, r00, r10, r01, r11,
                                                                szc_e[qe], szc_s[qe])
                                     : edge_emf_zcarry<1, false>(g, F, ii, jj, kk, r00, r10, r01, r11,
                                                                 szc_e[qe], szc_s[qe]);
            }
        }
    };
    // two barriers per plane: (1) E_z of plane k and E_x / E_y of plane
    // k + 1/2 as one flat loop (reads the reference EMFs of planes k, k + 1);
    // (2) the update of plane k, then the reference EMFs of plane k + 2 into
    // the slot of plane k, which (1) no longer reads
    int lo = 0;
    stage_ref(k0 - 1);
    stage_ref(k0);
    __syncthreads();
    for (int q = threadIdx.x; q < NEX + NEY; q += (TX * TY)) horizontal_edge(q, k0, lo, true);
    __syncthreads();
    stage_ref(k0 + 1);  // into the slot of plane k0 - 1, no longer read
    __syncthreads();
    bool bad = false;
    double mcfl = 0.0;
    uint32_t stcfl = 0;
    // the cell's z-face fluxes and (DT) base B_z at its low face k, read at k0
    // and carried up from the high face of the plane below
    const bool owner = i < ex && j < ey && i < nx && j < ny;
    double fzc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double bzc = 0.0;
    if (owner) {
        const idx_t fz0 = fidx(g, 2, i, j, k0);
#pragma unroll
        for (int q = 0; q < 5; ++q) fzc[q] = F.f[2][q][fz0];
        if (DT) bzc = base.b[2][face_store(g, 2, i, j, k0)];
    }
    for (int k = k0; k < k1; ++k) {
        const int sk = slot(k);
        for (int q = threadIdx.x; q < NEZ + NEX + NEY; q += (TX * TY)) {
            if (q < NEZ) {
                const int a = q % (TX + 1), c = q / (TX + 1), ii = i0 + a, jj = j0 + c;
                // E_z at (ii - 1/2, jj - 1/2, k): B = x, C = y
                if (ii <= nx && jj <= ny)
                    sez[c][a] = edge_emf<2>(g, F, ii, jj, k, sref[sk][2][c + 1][a + 1],
                                            sref[sk][2][c + 1][a], sref[sk][2][c][a + 1],
                                            sref[sk][2][c][a]);
            } else {
                horizontal_edge(q - NEZ, k + 1, 1 - lo, false);
            }
        }
        __syncthreads();
        const int hi = 1 - lo;
        double bzn = 0.0;
        if (i < ex && j < ey) {
            if (i < nx && j < ny) {
                const idx_t c = cell_store(g, i, j, k);
                const idx_t fx0 = fidx(g, 0, i, j, k), fx1 = fidx(g, 0, i + 1, j, k);
                const idx_t fy0 = fidx(g, 1, i, j, k), fy1 = fidx(g, 1, i, j + 1, k);
                const idx_t fz1 = fidx(g, 2, i, j, k + 1);
                double fzn[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) fzn[q] = F.f[2][q][fz1];
                const double dxr = F.f[0][0][fx1] - F.f[0][0][fx0];
                const double dyr = F.f[1][0][fy1] - F.f[1][0][fy0];
                const double dzr = fzn[0] - fzc[0];
                const double dxe = F.f[0][4][fx1] - F.f[0][4][fx0];
                const double dye = F.f[1][4][fy1] - F.f[1][4][fy0];
                const double dze = fzn[4] - fzc[4];
                const double dxmx = F.f[0][1][fx1] - F.f[0][1][fx0];
                const double dxmy = F.f[0][2][fx1] - F.f[0][2][fx0];
                const double dxmz = F.f[0][3][fx1] - F.f[0][3][fx0];
                const double dymy = F.f[1][1][fy1] - F.f[1][1][fy0];
                const double dymz = F.f[1][2][fy1] - F.f[1][2][fy0];
                const double dymx = F.f[1][3][fy1] - F.f[1][3][fy0];
                const double dzmz = fzn[1] - fzc[1];
                const double dzmx = fzn[2] - fzc[2];
                const double dzmy = fzn[3] - fzc[3];
#pragma unroll
                for (int q = 0; q < 5; ++q) fzc[q] = fzn[q];
                const double u0 = base.u[0][c] - cx * dxr - cy * dyr - cz * dzr;
                const double u1 = base.u[1][c] - cx * dxmx - cy * dymx - cz * dzmx;
                const double u2 = base.u[2][c] - cx * dxmy - cy * dymy - cz * dzmy;
                const double u3 = base.u[3][c] - cx * dxmz - cy * dymz - cz * dzmz;
                const double u4 = base.u[4][c] - cx * dxe - cy * dye - cz * dze;
                out.u[0][c] = u0;
                out.u[1][c] = u1;
                out.u[2][c] = u2;
                out.u[3][c] = u3;
                out.u[4][c] = u4;
                if (FULL) bad |= !isfinite(u0) || !isfinite(u1) || !isfinite(u2) || !isfinite(u3) ||
                                 !isfinite(u4);
                if (DT) {
                    // faces (i, j, k) low and high of the updated cell (a periodic
                    // high face through the face map, as its owner computes it)
                    const double bx0 = base.b[0][face_store(g, 0, i, j, k)]
                                       - cy * (sez[ty + 1][tx] - sez[ty][tx])
                                       + cz * (sey[hi][ty][tx] - sey[lo][ty][tx]);
                    const double bx1 = base.b[0][face_store(g, 0, map_face(i + 1, nx, g.bc[0]), j, k)]
                                       - cy * (sez[ty + 1][tx + 1] - sez[ty][tx + 1])
                                       + cz * (sey[hi][ty][tx + 1] - sey[lo][ty][tx + 1]);
                    const double by0 = base.b[1][face_store(g, 1, i, j, k)]
                                       - cz * (sex[hi][ty][tx] - sex[lo][ty][tx])
                                       + cx * (sez[ty][tx + 1] - sez[ty][tx]);
                    const double by1 = base.b[1][face_store(g, 1, i, map_face(j + 1, ny, g.bc[1]), k)]
                                       - cz * (sex[hi][ty + 1][tx] - sex[lo][ty + 1][tx])
                                       + cx * (sez[ty + 1][tx + 1] - sez[ty + 1][tx]);
                    const double bz0 = bzc
                                       - cx * (sey[lo][ty][tx + 1] - sey[lo][ty][tx])
                                       + cy * (sex[lo][ty + 1][tx] - sex[lo][ty][tx]);
                    bzn = base.b[2][face_store(g, 2, i, j, map_face(k + 1, nz, g.bc[2]))];
                    const double bz1 = bzn
                                       - cx * (sey[hi][ty][tx + 1] - sey[hi][ty][tx])
                                       + cy * (sex[hi][ty + 1][tx] - sex[hi][ty][tx]);
                    const double bcc[3] = {0.5 * (bx0 + bx1), 0.5 * (by0 + by1), 0.5 * (bz0 + bz1)};
                    mcfl = fmax(mcfl, cell_cfl(g, u0, u1, u2, u3, u4, bcc, stcfl));
                }
            }
            if (j < ny) {  // face x (i-1/2, j, k)
                const double b0 = base.b[0][face_store(g, 0, i, j, k)];
                const double v = b0 - cy * (sez[ty + 1][tx] - sez[ty][tx])
                                 + cz * (sey[hi][ty][tx] - sey[lo][ty][tx]);
                out.b[0][face_store(g, 0, i, j, k)] = v;
                if (g.bc[0] == VLCT_BC_PERIODIC && i == 0) out.b[0][face_store(g, 0, nx, j, k)] = v;
                if (FULL) bad |= !isfinite(v);
            }
            if (i < nx) {  // face y (i, j-1/2, k)
                const double b0 = base.b[1][face_store(g, 1, i, j, k)];
                const double v = b0 - cz * (sex[hi][ty][tx] - sex[lo][ty][tx])
                                 + cx * (sez[ty][tx + 1] - sez[ty][tx]);
                out.b[1][face_store(g, 1, i, j, k)] = v;
                if (g.bc[1] == VLCT_BC_PERIODIC && j == 0) out.b[1][face_store(g, 1, i, ny, k)] = v;
                if (FULL) bad |= !isfinite(v);
            }
            if (i < nx && j < ny) {  // face z (i, j, k-1/2)
                const double b0 = DT ? bzc : base.b[2][face_store(g, 2, i, j, k)];
                const double v = b0 - cx * (sey[lo][ty][tx + 1] - sey[lo][ty][tx])
                                 + cy * (sex[lo][ty + 1][tx] - sex[lo][ty][tx]);
                out.b[2][face_store(g, 2, i, j, k)] = v;
                if (g.bc[2] == VLCT_BC_PERIODIC && k == 0) out.b[2][face_store(g, 2, i, j, nz)] = v;
                if (FULL) bad |= !isfinite(v);
                if (DT) bzc = bzn;
            }
        }
        if (k + 2 <= k1) stage_ref(k + 2);
        __syncthreads();
        lo = hi;
    }
    // the top z faces of an outflow axis, from the last plane of edges
    if (k1 == nz && g.bc[2] == VLCT_BC_OUTFLOW && i < nx && j < ny && i < ex && j < ey) {
        const double b0 = base.b[2][face_store(g, 2, i, j, nz)];
        const double v = b0 - cx * (sey[lo][ty][tx + 1] - sey[lo][ty][tx])
                         + cy * (sex[lo][ty + 1][tx] - sex[lo][ty][tx]);
        out.b[2][face_store(g, 2, i, j, nz)] = v;
        if (FULL) bad |= !isfinite(v);
    }
    if (FULL && bad && status) atomicOr(status, kStatusNonfinite);
    if (DT) {
        if (stcfl && status) atomicOr(status, stcfl);
        __shared__ double red[(TX * TY) / 64];
        const double m = wave_max(mcfl);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            double r = red[0];
            for (int q = 1; q < (TX * TY) / 64; ++q) r = fmax(r, red[q]);
            partial[b] = r;
        }
    }
}

// ---------------------------------------------------------------------------
// fused predictor (Steps 2-5 in one kernel): the (column tile, plane) pairs
// of the grid, in z slabs, are dealt out to the blocks in equal shares
// (Geom::pred_slab, Geom::pred_chunk: one (slab, tile) per block, or a single
// slab shared out evenly over one wave of resident blocks); a block marches
// along z through each run [k0, k1) of planes of a TX x TY column tile that
// its share holds.  Per new plane m it
//   (A) derives the primitives of the tile plus a one-cell ring (Sec. 2.1,
//       B_cc = face average, floors) and the reference field -(v x B),
//   (B) solves PCM HLLD on the x- and y-faces of plane m and the z-face
//       m - 1/2 (Steps 2-3; every thread owns one column and the faces on its
//       low sides), keeping the hydro fluxes in registers and the face EMFs
//       and upwind indicators in LDS,
//   (C) forms the edge fields E_z of plane m and E_x, E_y of the half plane
//       m - 1/2 (Step 4, Eqs. emf-edge, emf-upwind-slope, emf-slope),
//   (D) updates the cells and the owned faces of plane m - 1 to t + dt/2
//       (Step 5).
// Nothing but U^n is read and nothing but U^{n+1/2} is written: primitives,
// fluxes and edge fields stay on chip.  For each run the block also
// evaluates the faces of the planes k0 - 1 and k1 (the edges of its first and
// last half planes need them).  Arithmetic per quantity is that of k_prims,
// k_flux and k_ct_update, whatever the runs.
// ---------------------------------------------------------------------------
template <int TX, int TY>
struct PredShape {
    static constexpr int CX = TX + 2, CY = TY + 2, NC = CX * CY;  // columns with the ring
    static constexpr int NT = (NC + 63) / 64 * 64;                  // threads (whole waves)
    static constexpr int NEZ = (TY + 1) * (TX + 1), NEX = (TY + 1) * TX, NEY = TY * (TX + 1);
};

// edge field from its four face EMFs, their upwind indicators and the four
// reference fields around the edge (the arithmetic of edge_emf)
__device__ __forceinline__ double edge_value(double eb_c, double eb_cm, double ec_b, double ec_bm,
                                             double sb_c, double sb_cm, double sc_b, double sc_bm,
                                             double r00, double r10, double r01, double r11)
{
    const double avg = 0.25 * (eb_c + eb_cm + ec_b + ec_bm);
    const double t1 = upwind(sb_c, ec_bm - r10, ec_b - r00);
    const double t2 = upwind(sb_cm, ec_bm - r11, ec_b - r01);
    const double t3 = upwind(sc_b, eb_cm - r01, eb_c - r00);
    const double t4 = upwind(sc_bm, eb_cm - r11, eb_c - r10);
    return avg + 0.25 * (t1 + t2 + t3 + t4);
}

// side0..2 (optional): the upwind side of every interior face, tape layout;
// P (optional, P.w[0] == NULL skips it): the half-step primitives of the
// interior cells are written there as k_prims would derive them from
// U^{n+1/2}; its ghost layers are left to k_prims_ghost.  Both are run-time
// choices of one kernel, so a taped step runs the very code of a plain one.
// ONE_RUN: block b is the single run of tile b mod ntiles in z slab
// b / ntiles (Geom::pred_chunk == 0); else its share of Geom::pred_chunk
// pairs in slab order (a zero chunk taken as one slab's worth).
template <int TX, int TY, bool ONE_RUN>
__device__ __forceinline__ void pred_body(const Geom &g, const StateP &s, const StateW &out,
                                          const Prims &P, const double *dt_dev, uint32_t *status,
                                          idx_t b, uint8_t *side0, uint8_t *side1, uint8_t *side2)
{
    using S = PredShape<TX, TY>;
    constexpr int CX = S::CX, CY = S::CY, NC = S::NC;
    constexpr int NEZ = S::NEZ, NEX = S::NEX, NEY = S::NEY;
    // W of the newest plane (8 primitives) and the hydro fluxes of the plane
    // being updated (x: 0-4, y: 5-9).  ONE_RUN keeps them apart (155 KB of
    // LDS in all), so that the next plane's primitives can be written while
    // the update still reads the fluxes and the barrier closing each plane
    // goes; the share form (a run loop, more registers) keeps both in s_wh
    // and the barrier, which measured faster there.
    __shared__ double s_pr[ONE_RUN ? 8 : 1][ONE_RUN ? NC : 1];
    __shared__ double s_wh[10][NC];
    auto PR = [&](int q, int c) -> double & {
        if constexpr (ONE_RUN) return s_pr[q][c];
        else return s_wh[q][c];
    };
    // reference fields: x and y components of the two newest planes (slot =
    // plane & 1), z component of the newest plane
    __shared__ double s_rx[2][NC], s_ry[2][NC], s_rz[NC];
    // face EMFs of the x- and y-faces of the two newest planes: x-face -F[B_y]
    // (E_z) and F[B_z] (E_y), y-face -F[B_z] (E_x) and F[B_x] (E_z)
    __shared__ double s_em[2][4][NC];
    __shared__ int8_t s_sg[2][2][NC];
    // z-face m - 1/2: -F[B_x] (E_y), F[B_y] (E_x) and its upwind indicator
    __shared__ double s_zem[2][NC];
    __shared__ int8_t s_zsg[NC];
    // edge fields: E_z of the planes, E_x / E_y of the half planes (slot = index & 1)
    __shared__ double s_ez[2][TY + 1][TX + 1];
    __shared__ double s_ex[2][TY + 1][TX];
    __shared__ double s_ey[2][TY][TX + 1];

    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int ex = nx + (g.bc[0] == VLCT_BC_OUTFLOW), ey = ny + (g.bc[1] == VLCT_BC_OUTFLOW);
    // the block's share: positions [pos0, pos1) of the sequence of (column
    // tile, plane) pairs ordered by z slab of Geom::pred_slab planes (the last
    // slab holds the remainder), then tile, then plane; it marches each run of
    // one tile's planes in turn
    const int ntx = (ex + TX - 1) / TX, nty = (ey + TY - 1) / TY, ntiles = ntx * nty;
    const int npos = ntiles * nz;  // below 2^31 for sides up to kMaxN
    const int H = g.pred_slab, nfull = nz / H, rem = nz - nfull * H;
    if (ONE_RUN && b >= (idx_t)ntiles * (nfull + (rem > 0))) return;
    const int chunk = g.pred_chunk > 0 ? g.pred_chunk : H;
    if (!ONE_RUN && b * (idx_t)chunk >= npos) return;
    const double dt = 0.5 * dt_dev[0];
    const double cx = dt / g.dl[0], cy = dt / g.dl[1], cz = dt / g.dl[2];

    // this thread's column: (a, c) in the tile with its ring
    const int t = threadIdx.x;
    const bool col = t < NC;
    const int a = t % CX, c = t / CX;
    const int tx = a - 1, ty = c - 1;
    uint32_t st = 0;
    auto run = [&](const int tile, const int k0, const int k1) {
        const int i0 = (tile % ntx) * TX, j0 = (tile / ntx) * TY;
        // cell (ii, jj) of the column
        const int ii = i0 - 1 + a, jj = j0 - 1 + c;
        const bool live = col && ii <= nx && jj <= ny;
        const bool do_x = live && a >= 1, do_y = live && c >= 1;
        const bool do_z = live && !((a == 0 || a == CX - 1) && (c == 0 || c == CY - 1));
        // owned positions: cells / faces of the tile proper
        const bool own = live && a >= 1 && a <= TX && c >= 1 && c <= TY && ii < ex && jj < ey;
        const bool interior = own && ii < nx && jj < ny;
        const int mi = map_cell(ii, nx, g.bc[0]), mj = map_cell(jj, ny, g.bc[1]);
        const int fi0 = map_face(ii, nx, g.bc[0]), fi1 = map_face(ii + 1, nx, g.bc[0]);
        const int fj0 = map_face(jj, ny, g.bc[1]), fj1 = map_face(jj + 1, ny, g.bc[1]);

        W7 wz_prev{};                   // own cell of the previous plane, z sweep frame
        double hx[5] = {}, hy[5] = {};  // own x-, y-face hydro fluxes of the previous plane
        double hz_lo[5] = {};           // own z-face hydro flux below the previous plane

        // U^n of this thread's cell in a plane: 5 conserved values and the six faces
        double pf[11];
        auto load_plane = [&](int m) {
            const int mk = map_cell(m, nz, g.bc[2]);
            const idx_t cc = cell_store(g, mi, mj, mk);
#pragma unroll
            for (int q = 0; q < 5; ++q) pf[q] = s.u[q][cc];
            pf[5] = s.b[0][face_store(g, 0, fi0, mj, mk)];
            pf[6] = s.b[0][face_store(g, 0, fi1, mj, mk)];
            pf[7] = s.b[1][face_store(g, 1, mi, fj0, mk)];
            pf[8] = s.b[1][face_store(g, 1, mi, fj1, mk)];
            pf[9] = s.b[2][face_store(g, 2, mi, mj, map_face(m, nz, g.bc[2]))];
            pf[10] = s.b[2][face_store(g, 2, mi, mj, map_face(m + 1, nz, g.bc[2]))];
        };

        for (int m = k0 - 1; m <= k1; ++m) {
            const int sm = m & 1, sp = sm ^ 1;
            // (A) primitives and reference field of plane m; the cell's low faces
            // are also the normal fields of the faces this thread solves in (B)
            double bx0 = 0.0, by0 = 0.0, bz0 = 0.0;
            if (live) {
                load_plane(m);
                bx0 = pf[5];
                const double bx1 = pf[6];
                by0 = pf[7];
                const double by1 = pf[8];
                bz0 = pf[9];
                const double bz1 = pf[10];
                const double bcx = 0.5 * (bx0 + bx1);
                const double bcy = 0.5 * (by0 + by1);
                const double bcz = 0.5 * (bz0 + bz1);
                double d = pf[0];
                if (!(d >= kFloorRho)) { d = kFloorRho; st |= kStatusDensityFloor; }
                const double id = 1.0 / d;
                const double vx = pf[1] * id, vy = pf[2] * id, vz = pf[3] * id;
                const double ke = 0.5 * d * (vx * vx + vy * vy + vz * vz);
                const double me = 0.5 * (bcx * bcx + bcy * bcy + bcz * bcz);
                double pr = (g.gamma - 1.0) * (pf[4] - ke - me);
                if (!(pr >= kFloorP)) { pr = kFloorP; st |= kStatusPressureFloor; }
                PR(0, t) = d;
                PR(1, t) = vx;
                PR(2, t) = vy;
                PR(3, t) = vz;
                PR(4, t) = pr;
                PR(5, t) = bcx;
                PR(6, t) = bcy;
                PR(7, t) = bcz;
                s_rx[sm][t] = -(vy * bcz - vz * bcy);
                s_ry[sm][t] = -(vz * bcx - vx * bcz);
                s_rz[t] = -(vx * bcy - vy * bcx);
            }
            __syncthreads();
            // (B) PCM HLLD on the x-, y-faces of plane m and the z-face m - 1/2
            double hxn[5] = {}, hyn[5] = {}, hzn[5] = {};
            W7 wz{};
            if (live) {
                const W7 wxr{PR(0, t), PR(1, t), PR(2, t), PR(3, t), PR(4, t), PR(6, t), PR(7, t)};
                wz = W7{PR(0, t), PR(3, t), PR(1, t), PR(2, t), PR(4, t), PR(5, t), PR(6, t)};
                double f[7], upw;
                if (do_x) {
                    const int l = t - 1;
                    const W7 wl{PR(0, l), PR(1, l), PR(2, l), PR(3, l), PR(4, l), PR(6, l), PR(7, l)};
                    hlld(wl, wxr, bx0, g.gamma, g.gm1i, f, upw);
#pragma unroll
                    for (int q = 0; q < 5; ++q) hxn[q] = f[q];
                    s_em[sm][0][t] = -f[5];
                    s_em[sm][1][t] = f[6];
                    s_sg[sm][0][t] = (int8_t)upw;
                }
                if (do_y) {
                    const int l = t - CX;
                    const W7 wl{PR(0, l), PR(2, l), PR(3, l), PR(1, l), PR(4, l), PR(7, l), PR(5, l)};
                    const W7 wr{PR(0, t), PR(2, t), PR(3, t), PR(1, t), PR(4, t), PR(7, t), PR(5, t)};
                    hlld(wl, wr, by0, g.gamma, g.gm1i, f, upw);
#pragma unroll
                    for (int q = 0; q < 5; ++q) hyn[q] = f[q];
                    s_em[sm][2][t] = -f[5];
                    s_em[sm][3][t] = f[6];
                    s_sg[sm][1][t] = (int8_t)upw;
                }
                if (do_z && m >= k0) {
                    hlld(wz_prev, wz, bz0, g.gamma, g.gm1i, f, upw);
#pragma unroll
                    for (int q = 0; q < 5; ++q) hzn[q] = f[q];
                    s_zem[0][t] = -f[5];
                    s_zem[1][t] = f[6];
                    s_zsg[t] = (int8_t)upw;
                }
            }
            __syncthreads();
            // (C) E_z of plane m, E_x / E_y of the half plane m - 1/2; the hydro
            // fluxes of plane m - 1 go to LDS for the neighbours' updates.  The
            // U^n values the update of plane m - 1 in (D) starts from are loaded
            // first, so that their latency hides behind the edge computations.
            const bool upd = m - 1 >= k0 && m - 1 < k1;
            double u0[5] = {}, bxb = 0.0, byb = 0.0, bzb = 0.0, bxh = 0.0, byh = 0.0, bzh = 0.0;
            if (upd && own) {
                const int k = m - 1;
                if (interior) {
                    const idx_t cc = cell_store(g, ii, jj, k);
#pragma unroll
                    for (int q = 0; q < 5; ++q) u0[q] = s.u[q][cc];
                    bzb = s.b[2][face_store(g, 2, ii, jj, k)];
                    if (P.w[0]) {
                        bxh = s.b[0][face_store(g, 0, map_face(ii + 1, nx, g.bc[0]), jj, k)];
                        byh = s.b[1][face_store(g, 1, ii, map_face(jj + 1, ny, g.bc[1]), k)];
                        bzh = s.b[2][face_store(g, 2, ii, jj, map_face(k + 1, nz, g.bc[2]))];
                    }
                }
                if (jj < ny) bxb = s.b[0][face_store(g, 0, ii, jj, k)];
                if (ii < nx) byb = s.b[1][face_store(g, 1, ii, jj, k)];
            }
            if (m >= k0) {
                const int nez = m < k1 ? NEZ : 0;
                for (int q = threadIdx.x; q < nez + NEX + NEY; q += S::NT) {
                    if (q < nez) {
                        const int ea = q % (TX + 1), ec = q / (TX + 1), ie = i0 + ea, je = j0 + ec;
                        // E_z at (ie - 1/2, je - 1/2, m): B = x-faces, C = y-faces
                        if (ie <= nx && je <= ny) {
                            const int o = (ec + 1) * CX + ea + 1;  // column (ie, je)
                            s_ez[sm][ec][ea] = edge_value(
                                s_em[sm][0][o], s_em[sm][0][o - CX], s_em[sm][3][o], s_em[sm][3][o - 1],
                                s_sg[sm][0][o], s_sg[sm][0][o - CX], s_sg[sm][1][o], s_sg[sm][1][o - 1],
                                s_rz[o], s_rz[o - 1], s_rz[o - CX], s_rz[o - CX - 1]);
                        }
                    } else if (q < nez + NEX) {
                        const int r = q - nez;
                        const int ea = r % TX, ec = r / TX, ie = i0 + ea, je = j0 + ec;
                        // E_x at (ie, je - 1/2, m - 1/2): B = y-faces (planes m, m - 1), C = z-faces
                        if (ie < nx && je <= ny) {
                            const int o = (ec + 1) * CX + ea + 1;
                            s_ex[sm][ec][ea] = edge_value(
                                s_em[sm][2][o], s_em[sp][2][o], s_zem[1][o], s_zem[1][o - CX],
                                s_sg[sm][1][o], s_sg[sp][1][o], s_zsg[o], s_zsg[o - CX],
                                s_rx[sm][o], s_rx[sm][o - CX], s_rx[sp][o], s_rx[sp][o - CX]);
                        }
                    } else {
                        const int r = q - nez - NEX;
                        const int ea = r % (TX + 1), ec = r / (TX + 1), ie = i0 + ea, je = j0 + ec;
                        // E_y at (ie - 1/2, je, m - 1/2): B = z-faces, C = x-faces (planes m, m - 1)
                        if (ie <= nx && je < ny) {
                            const int o = (ec + 1) * CX + ea + 1;
                            s_ey[sm][ec][ea] = edge_value(
                                s_zem[0][o], s_zem[0][o - 1], s_em[sm][1][o], s_em[sp][1][o],
                                s_zsg[o], s_zsg[o - 1], s_sg[sm][0][o], s_sg[sp][0][o],
                                s_ry[sm][o], s_ry[sp][o], s_ry[sm][o - 1], s_ry[sp][o - 1]);
                        }
                    }
                }
            }
            if (upd && live) {
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    s_wh[q][t] = hx[q];
                    s_wh[5 + q][t] = hy[q];
                }
            }
            // the tape: upwind sides of the interior cell's low faces in plane m
            if (side0 && interior && m >= k0 && m < k1) {
                const idx_t cc = cell_store(g, ii, jj, m);
                side0[cc] = side_code(s_sg[sm][0][t]);
                side1[cc] = side_code(s_sg[sm][1][t]);
                side2[cc] = side_code(s_zsg[t]);
            }
            __syncthreads();
            // (D) half-step update of plane k = m - 1 (Step 5); an interior cell
            // also derives its half-step primitives (for the corrector), with its
            // high faces recomputed from the same edge fields and in the same
            // arithmetic as the threads or blocks that own them
            if (upd && own) {
                const int k = m - 1;
                const int lo = sp, hi = sm;  // half planes k - 1/2 and k + 1/2
                const int ke = k & 1;        // E_z slot of plane k
                double u[5] = {}, bxl = 0.0, byl = 0.0, bzl = 0.0;
                if (interior) {
                    const idx_t cc = cell_store(g, ii, jj, k);
                    const double dxr = s_wh[0][t + 1] - hx[0];
                    const double dyr = s_wh[5][t + CX] - hy[0];
                    const double dzr = hzn[0] - hz_lo[0];
                    const double dxe = s_wh[4][t + 1] - hx[4];
                    const double dye = s_wh[9][t + CX] - hy[4];
                    const double dze = hzn[4] - hz_lo[4];
                    const double dxmx = s_wh[1][t + 1] - hx[1];
                    const double dxmy = s_wh[2][t + 1] - hx[2];
                    const double dxmz = s_wh[3][t + 1] - hx[3];
                    const double dymy = s_wh[6][t + CX] - hy[1];
                    const double dymz = s_wh[7][t + CX] - hy[2];
                    const double dymx = s_wh[8][t + CX] - hy[3];
                    const double dzmz = hzn[1] - hz_lo[1];
                    const double dzmx = hzn[2] - hz_lo[2];
                    const double dzmy = hzn[3] - hz_lo[3];
                    u[0] = u0[0] - cx * dxr - cy * dyr - cz * dzr;
                    u[1] = u0[1] - cx * dxmx - cy * dymx - cz * dzmx;
                    u[2] = u0[2] - cx * dxmy - cy * dymy - cz * dzmy;
                    u[3] = u0[3] - cx * dxmz - cy * dymz - cz * dzmz;
                    u[4] = u0[4] - cx * dxe - cy * dye - cz * dze;
#pragma unroll
                    for (int q = 0; q < 5; ++q) out.u[q][cc] = u[q];
                }
                if (jj < ny) {  // face x (ii - 1/2, jj, k)
                    const double v = bxb - cy * (s_ez[ke][ty + 1][tx] - s_ez[ke][ty][tx])
                                     + cz * (s_ey[hi][ty][tx] - s_ey[lo][ty][tx]);
                    out.b[0][face_store(g, 0, ii, jj, k)] = v;
                    if (g.bc[0] == VLCT_BC_PERIODIC && ii == 0) out.b[0][face_store(g, 0, nx, jj, k)] = v;
                    bxl = v;
                }
                if (ii < nx) {  // face y (ii, jj - 1/2, k)
                    const double v = byb - cz * (s_ex[hi][ty][tx] - s_ex[lo][ty][tx])
                                     + cx * (s_ez[ke][ty][tx + 1] - s_ez[ke][ty][tx]);
                    out.b[1][face_store(g, 1, ii, jj, k)] = v;
                    if (g.bc[1] == VLCT_BC_PERIODIC && jj == 0) out.b[1][face_store(g, 1, ii, ny, k)] = v;
                    byl = v;
                }
                if (interior) {  // face z (ii, jj, k - 1/2)
                    const double v = bzb - cx * (s_ey[lo][ty][tx + 1] - s_ey[lo][ty][tx])
                                     + cy * (s_ex[lo][ty + 1][tx] - s_ex[lo][ty][tx]);
                    out.b[2][face_store(g, 2, ii, jj, k)] = v;
                    if (g.bc[2] == VLCT_BC_PERIODIC && k == 0) out.b[2][face_store(g, 2, ii, jj, nz)] = v;
                    bzl = v;
                }
                if (interior && P.w[0]) {
                    // high faces (a periodic one through the face map, as its owner computes it)
                    const double bxu = bxh - cy * (s_ez[ke][ty + 1][tx + 1] - s_ez[ke][ty][tx + 1])
                                       + cz * (s_ey[hi][ty][tx + 1] - s_ey[lo][ty][tx + 1]);
                    const double byu = byh - cz * (s_ex[hi][ty + 1][tx] - s_ex[lo][ty + 1][tx])
                                       + cx * (s_ez[ke][ty + 1][tx + 1] - s_ez[ke][ty + 1][tx]);
                    const double bzu = bzh - cx * (s_ey[hi][ty][tx + 1] - s_ey[hi][ty][tx])
                                       + cy * (s_ex[hi][ty + 1][tx] - s_ex[hi][ty][tx]);
                    st |= prims_store(g, P, pidx(g, ii, jj, k), u, 0.5 * (bxl + bxu), 0.5 * (byl + byu),
                                      0.5 * (bzl + bzu));
                }
            }
            // the top z faces of an outflow axis, from the edges of the half plane nz - 1/2
            if (m == k1 && k1 == nz && g.bc[2] == VLCT_BC_OUTFLOW && interior) {
                const double b0 = s.b[2][face_store(g, 2, ii, jj, nz)];
                const double v = b0 - cx * (s_ey[sm][ty][tx + 1] - s_ey[sm][ty][tx])
                                 + cy * (s_ex[sm][ty + 1][tx] - s_ex[sm][ty][tx]);
                out.b[2][face_store(g, 2, ii, jj, nz)] = v;
            }
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                hx[q] = hxn[q];
                hy[q] = hyn[q];
                hz_lo[q] = hzn[q];
            }
            wz_prev = wz;
            // ONE_RUN needs no barrier here: the next plane's (A) writes only
            // s_pr and the reference fields, which (D) does not read, and
            // everything (D) reads is next written after the barrier that
            // closes (A)
            if (!ONE_RUN) __syncthreads();
        }
    };
    if (ONE_RUN) {
        const int tile = (int)(b % ntiles), sl = (int)(b / ntiles);
        run(tile, sl * H, min(sl * H + H, nz));
    } else {
        const int pos0 = (int)b * chunk, pos1 = min(pos0 + chunk, npos);
        const int fullpos = nfull * ntiles * H;
        for (int pos = pos0; pos < pos1;) {
            int tile, k0, len;
            if (pos < fullpos) {
                const int sl = pos / (ntiles * H), r = pos - sl * ntiles * H;
                tile = r / H;
                const int kk = r - tile * H;
                k0 = sl * H + kk;
                len = H - kk;
            } else {
                const int r = pos - fullpos;
                tile = r / rem;
                const int kk = r - tile * rem;
                k0 = nfull * H + kk;
                len = rem - kk;
            }
            const int k1 = k0 + min(len, pos1 - pos);
            pos += k1 - k0;
            run(tile, k0, k1);
        }
    }
    if (st && status) atomicOr(status, st);
}

// ---------------------------------------------------------------------------
// CFL reduction (Step 1, Eq. dt): per-block maxima of max_l (|v_l| + c_f,l)/d_l,
// then one block reduces the partials and writes dt = cfl / max.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dt_partial_body(const Geom &g, const StateP &s, double *partial,
                                                uint32_t *status, idx_t b)
{
    __shared__ double red[kBlock / 64];
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = b * kBlock + threadIdx.x;
    double m = 0.0;
    if (t < N) {
        const int i = (int)(t % g.n[0]);
        const idx_t r = t / g.n[0];
        const int j = (int)(r % g.n[1]);
        const int k = (int)(r / g.n[1]);
        // high faces through the face map: a periodic duplicate face is not read
        const int ip = map_face(i + 1, g.n[0], g.bc[0]);
        const int jp = map_face(j + 1, g.n[1], g.bc[1]);
        const int kp = map_face(k + 1, g.n[2], g.bc[2]);
        const double b[3] = {
            0.5 * (s.b[0][face_store(g, 0, i, j, k)] + s.b[0][face_store(g, 0, ip, j, k)]),
            0.5 * (s.b[1][face_store(g, 1, i, j, k)] + s.b[1][face_store(g, 1, i, jp, k)]),
            0.5 * (s.b[2][face_store(g, 2, i, j, k)] + s.b[2][face_store(g, 2, i, j, kp)])};
        uint32_t st = 0;
        m = cell_cfl(g, s.u[0][t], s.u[1][t], s.u[2][t], s.u[3][t], s.u[4][t], b, st);
        if (st && status) atomicOr(status, st);
    }
    m = wave_max(m);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double red_max = red[0];
        for (int q = 1; q < kBlock / 64; ++q) red_max = fmax(red_max, red[q]);
        partial[b] = red_max;
    }
}

__global__ void __launch_bounds__(1024) k_dt_final(const double *partial, int n, double cfl,
                                                   double *dt_out)
{
    __shared__ double red[1024 / 64];
    double m = 0.0;
    for (int q = threadIdx.x; q < n; q += blockDim.x) m = fmax(m, partial[q]);
    m = wave_max(m);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = red[0];
        for (int q = 1; q < (int)(blockDim.x / 64); ++q) b = fmax(b, red[q]);
        dt_out[0] = cfl / b;
    }
}

// ---------------------------------------------------------------------------
// single-instance kernels: the logical block comes from the XCD remap
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_prims(Geom g, StateP s, Prims P, uint32_t *status)
{
    prims_body(g, s, P, status, xcd_block(nblk_prims(g)));
}

template <int D, int RECON>
__global__ void __launch_bounds__(kBlock) k_flux(Geom g, StateP s, Prims P, Flux F,
                                                 uint32_t *status)
{
    flux_pcm_body<D, RECON>(g, s, P, F, status, xcd_block(nblk_flux(g, D)));
}

template <int RECON>
__global__ void __launch_bounds__(kBlock) k_flux_recon_x(Geom g, StateP s, Prims P, Flux F,
                                                          uint32_t *status)
{
    recon_x_body<RECON>(g, s, P, F, status, xcd_block(nblk_row(g)));
}

template <int D, int RECON, int M = kMarch>
__global__ void __launch_bounds__(kBlock) k_flux_recon_march(Geom g, StateP s, Prims P, Flux F,
                                                              uint32_t *status)
{
    march_body<D, RECON, M>(g, s, P, F, status, xcd_block(nblk_march(g, D, M)));
}

// march segment of a single step's corrector: 16 faces, or 8 when the
// 16-face launch would have fewer than 1024 blocks (4 per CU)
static int march_segment(const Geom &g, int d)
{
    const int o = tile_override("march");
    if (o == 8 || o == kMarch) return o;
    return nblk_march(g, d, kMarch) < 1024 ? 8 : kMarch;
}

template <bool FULL, bool DT = false>
__global__ void __launch_bounds__(kCt, 4) k_ct_update(Geom g, Prims P, Flux F, StateP base,
                                                       StateW out, const double *dt_dev,
                                                       uint32_t *status, double *partial)
{
    ct_body<FULL, kTx, kTy, DT>(g, P, F, base, out, dt_dev, status, xcd_block(nblk_ct(g)),
                                partial);
}

constexpr int kPredThreads = PredShape<kPredTx, kPredTy>::NT;
static_assert(kPredThreads * kPredBlocksPerCU <= 1024,
              "the resident predictor blocks of a CU hold at most two waves per SIMD");

// blocks of the fused predictor: one per (slab, tile) (Geom::pred_chunk == 0),
// else shares of Geom::pred_chunk (tile, plane) pairs
__host__ __device__ __forceinline__ idx_t nblk_pred(const Geom &g)
{
    const idx_t nsl = (g.n[2] + g.pred_slab - 1) / g.pred_slab;
    if (g.pred_chunk == 0) return pred_tiles(g) * nsl;
    const idx_t npos = pred_tiles(g) * g.n[2];
    return (npos + g.pred_chunk - 1) / g.pred_chunk;
}
// blocks of the share form (the batched step's), a zero chunk taken as one slab
__host__ __device__ __forceinline__ idx_t nblk_pred_shares(const Geom &g)
{
    const idx_t npos = pred_tiles(g) * g.n[2];
    const idx_t chunk = g.pred_chunk > 0 ? g.pred_chunk : g.pred_slab;
    return (npos + chunk - 1) / chunk;
}

template <bool ONE_RUN>
__global__ void __launch_bounds__(kPredThreads, kPredWavesPerSimd) k_pred(Geom g, StateP s, StateW out, Prims P,
                                                        const double *dt_dev, uint32_t *status,
                                                        uint8_t *side0, uint8_t *side1,
                                                        uint8_t *side2)
{
    pred_body<kPredTx, kPredTy, ONE_RUN>(g, s, out, P, dt_dev, status, xcd_block(nblk_pred(g)),
                                         side0, side1, side2);
}

__global__ void __launch_bounds__(kBlock) k_prims_ghost(Geom g, StateP s, Prims P,
                                                        uint32_t *status)
{
    prims_ghost_body(g, s, P, status, xcd_block((ghost_cells(g) + kBlock - 1) / kBlock));
}

__global__ void __launch_bounds__(kBlock) k_dt_partial(Geom g, StateP s, double *partial,
                                                       uint32_t *status)
{
    dt_partial_body(g, s, partial, status, blockIdx.x);
}

// ---------------------------------------------------------------------------
// batched step: independent instances (own sizes, gamma, dt, boundaries,
// workspace) advanced by one launch per kernel for all of them.  Each launch
// flattens the logical blocks of every instance; a block finds its instance
// by binary search over the first block of each instance and runs the same
// body as the single-instance kernel, so an instance's result equals its
// single-instance step bit for bit.
// ---------------------------------------------------------------------------
// launches of a batched step; the march and CT launches come once per tile
// variant (an instance has blocks only in the slot of its own variant)
enum Slot {
    kSlotPred,
    kSlotGhost,
    kSlotPrims,
    kSlotFlux0,
    kSlotFlux1,
    kSlotFlux2,
    kSlotRow,
    kSlotMarch1,
    kSlotMarch2 = kSlotMarch1 + kMarchVariants,
    kSlotCt = kSlotMarch2 + kMarchVariants,
    kSlotDt = kSlotCt + kCtVariants,
    kSlots
};

struct Inst {
    Geom g;
    StateP in;       // U^n
    StateW out;      // U^{n+1}
    StateW half;     // U^{n+1/2} (workspace)
    Prims P;         // primitives of the current stage (workspace)
    Flux F;          // face fluxes of the current stage (workspace)
    double *partial; // CFL partials (workspace)
    const double *dt;
    double *next_dt;
    uint32_t *status;
    // per-instance end times (vlct_step_batch_until; NULL otherwise): the
    // instance steps only while *active, by *dt = min(caller dt, t_end - t),
    // and its time *t advances at the end of the step
    const int *active;
    double *t;
    idx_t start[kSlots];  // first flattened block of this instance in each launch
};

__device__ __forceinline__ bool retired(const Inst &I) { return I.active && !I.active[0]; }

constexpr int kPackChunk = 4;  // records per pack launch (kernel-argument size)
struct PackArgs {
    Inst rec[kPackChunk];
    Inst *tab;
    int first, n;
};

// writes instance records into the device table (records travel as kernel
// arguments, so a step needs no host-to-device copy and can be captured)
__global__ void k_pack(PackArgs a)
{
    const int t = threadIdx.x;
    if (t < a.n) a.tab[a.first + t] = a.rec[t];
}

__device__ __forceinline__ const Inst &find_inst(const Inst *tab, int count, int slot, idx_t gb,
                                                 idx_t &lb)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].start[slot] <= gb) lo = mid; else hi = mid - 1;
    }
    lb = gb - tab[lo].start[slot];
    return tab[lo];
}

__device__ __forceinline__ StateP const_view(const StateW &w)
{
    StateP p;
    for (int f = 0; f < 5; ++f) p.u[f] = w.u[f];
    for (int d = 0; d < 3; ++d) p.b[d] = w.b[d];
    return p;
}

// the fused predictor of every instance: U^n -> U^{n+1/2}
__global__ void __launch_bounds__(kPredThreads, kPredWavesPerSimd) kb_pred(const Inst *tab, int count, idx_t total)
{
    const idx_t gb = xcd_block(total);
    if (gb >= total) return;
    idx_t lb;
    const Inst &I = find_inst(tab, count, kSlotPred, gb, lb);
    if (retired(I)) return;
    const Geom g = I.g;
    const StateP in = I.in;
    const StateW half = I.half;
    const Prims P = I.P;
    pred_body<kPredTx, kPredTy, false>(g, in, half, P, I.dt, I.status, lb, nullptr, nullptr,
                                       nullptr);
}

// ghost-layer primitives of the half-step state of every instance
__global__ void __launch_bounds__(kBlock) kb_prims_ghost(const Inst *tab, int count, idx_t total)
{
    const idx_t gb = xcd_block(total);
    if (gb >= total) return;
    idx_t lb;
    const Inst &I = find_inst(tab, count, kSlotGhost, gb, lb);
    if (retired(I)) return;
    const Geom g = I.g;
    const StateP st = const_view(I.half);
    const Prims P = I.P;
    prims_ghost_body(g, st, P, I.status, lb);
}

// half = 0: primitives of U^n, 1: of U^{n+1/2}
__global__ void __launch_bounds__(kBlock) kb_prims(const Inst *tab, int count, idx_t total,
                                                   int half)
{
    const idx_t gb = xcd_block(total);
    if (gb >= total) return;
    idx_t lb;
    const Inst &I = find_inst(tab, count, kSlotPrims, gb, lb);
    if (retired(I)) return;
    const Geom g = I.g;
    const StateP st = half ? const_view(I.half) : I.in;
    const Prims P = I.P;
    prims_body(g, st, P, I.status, lb);
}

// half = 0: predictor on U^n, 1: PCM corrector on U^{n+1/2}
template <int D>
__global__ void __launch_bounds__(kBlock) kb_flux_pcm(const Inst *tab, int count, idx_t total,
                                                      int half)
{
    const idx_t gb = xcd_block(total);
    if (gb >= total) return;
    idx_t lb;
    const Inst &I = find_inst(tab, count, kSlotFlux0 + D, gb, lb);
    if (retired(I)) return;
    const Geom g = I.g;
    const StateP st = half ? const_view(I.half) : I.in;
    const Prims P = I.P;
    const Flux F = I.F;
    flux_pcm_body<D, VLCT_RECON_PCM>(g, st, P, F, I.status, lb);
}

template <int RECON>
__global__ void __launch_bounds__(kBlock) kb_recon_x(const Inst *tab, int count, idx_t total)
{
    const idx_t gb = xcd_block(total);
    if (gb >= total) return;
    idx_t lb;
    const Inst &I = find_inst(tab, count, kSlotRow, gb, lb);
    if (retired(I)) return;
    const Geom g = I.g;
    const StateP st = const_view(I.half);
    const Prims P = I.P;
    const Flux F = I.F;
    recon_x_body<RECON>(g, st, P, F, I.status, lb);
}

template <int D, int RECON, int V>
__global__ void __launch_bounds__(kBlock) kb_march(const Inst *tab, int count, idx_t total)
{
    const idx_t gb = xcd_block(total);
    if (gb >= total) return;
    idx_t lb;
    const Inst &I = find_inst(tab, count, (D == 1 ? kSlotMarch1 : kSlotMarch2) + V, gb, lb);
    if (retired(I)) return;
    const Geom g = I.g;
    const StateP st = const_view(I.half);
    const Prims P = I.P;
    const Flux F = I.F;
    march_body<D, RECON, march_len(V)>(g, st, P, F, I.status, lb);
}

template <bool FULL, int V>
__global__ void __launch_bounds__(kCt, 4) kb_ct(const Inst *tab, int count, idx_t total)
{
    const idx_t gb = xcd_block(total);
    if (gb >= total) return;
    idx_t lb;
    const Inst &I = find_inst(tab, count, kSlotCt + V, gb, lb);
    if (retired(I)) return;
    const Geom g = I.g;
    const Prims P = I.P;
    const Flux F = I.F;
    const StateP base = I.in;
    const StateW out = FULL ? I.out : I.half;
    ct_body<FULL, ct_tx(V), ct_ty(V)>(g, P, F, base, out, I.dt, I.status, lb);
}

__global__ void __launch_bounds__(kBlock) kb_dt_partial(const Inst *tab, int count, idx_t total)
{
    // no XCD remap: the partial of block lb is written to partial[lb]
    const idx_t gb = blockIdx.x;
    if (gb >= total) return;
    idx_t lb;
    const Inst &I = find_inst(tab, count, kSlotDt, gb, lb);
    if (retired(I)) return;
    const Geom g = I.g;
    dt_partial_body(g, const_view(I.out), I.partial, I.status, lb);
}

// one block per instance: dt = cfl / max over that instance's partials; an
// instance with an end time also advances its time by the step it took
__global__ void __launch_bounds__(1024) kb_dt_final(const Inst *tab)
{
    const Inst &I = tab[blockIdx.x];
    if (retired(I)) return;
    const int n = (int)nblk_dt(I.g);
    __shared__ double red[1024 / 64];
    double m = 0.0;
    for (int q = threadIdx.x; q < n; q += blockDim.x) m = fmax(m, I.partial[q]);
    m = wave_max(m);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = red[0];
        for (int q = 1; q < (int)(blockDim.x / 64); ++q) b = fmax(b, red[q]);
        I.next_dt[0] = I.g.cfl / b;
        if (I.t) I.t[0] += I.dt[0];
    }
}

// per-instance end times: instance i is active while t[i] < t_end[i] and then
// steps by min(dt[i], t_end[i] - t[i]) (the caller's clip of the last step)
__global__ void kb_clip(int count, const double *dt, const double *t, const double *t_end,
                        double *dt_eff, int *active)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const bool a = t[i] < t_end[i];
    active[i] = a ? 1 : 0;
    dt_eff[i] = a ? fmin(dt[i], t_end[i] - t[i]) : 0.0;
}

// ---------------------------------------------------------------------------
// host side: validation, workspace carving, launches
// ---------------------------------------------------------------------------




struct Layout {
    size_t half[8], prims, flux[3], partial, total;
    size_t prims_len, flux_len[3], npartial;
};

static Layout layout(const Geom &g)
{
    Layout L;
    size_t off = 0;
    for (int f = 0; f < 8; ++f) {
        L.half[f] = off;
        off += align_up(field_len(g.n, f) * sizeof(double));
    }
    L.prims_len = (size_t)g.p[0] * g.p[1] * g.p[2];
    L.prims = off;
    off += 8 * align_up(L.prims_len * sizeof(double));
    for (int d = 0; d < 3; ++d) {
        L.flux_len[d] = (size_t)flux_dim(g.n, d, 0) * flux_dim(g.n, d, 1) * flux_dim(g.n, d, 2);
        L.flux[d] = off;
        off += flux_axis_bytes(L.flux_len[d]);
    }
    const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    L.npartial = (N + kBlock - 1) / kBlock;  // partials of the CFL kernel
    L.partial = off;
    // room also for one partial per CT block (the CFL reduction fused into the full step)
    off += align_up(std::max<size_t>(L.npartial, (size_t)nblk_ct(g)) * sizeof(double));
    L.total = off;
    return L;
}


// launch observer of one vlct_step_observed call (diagnostics): set by that
// call on its own host thread for its duration only, so other calls and
// threads never see it
struct ObserverCtx {
    vlct_launch_observer cb;
    void *user;
};
static thread_local const ObserverCtx *t_observer = nullptr;

struct Observe {
    int kernel;
    hipStream_t s;
    Observe(int k, hipStream_t st) : kernel(k), s(st)
    {
        if (t_observer) t_observer->cb(t_observer->user, kernel, 0, static_cast<void *>(s));
    }
    ~Observe()
    {
        if (t_observer) t_observer->cb(t_observer->user, kernel, 1, static_cast<void *>(s));
    }
};

struct Bound {
    Prims P;
    Flux F;
    StateW half;
    double *partial;
};

static Bound bind(const Layout &L, void *ws)
{
    char *b = static_cast<char *>(ws);
    Bound B;
    for (int f = 0; f < 8; ++f) {
        double *p = reinterpret_cast<double *>(b + L.half[f]);
        if (f < 5) B.half.u[f] = p; else B.half.b[f - 5] = p;
    }
    for (int f = 0; f < 8; ++f)
        B.P.w[f] = reinterpret_cast<double *>(b + L.prims + f * align_up(L.prims_len * sizeof(double)));
    B.F = bind_flux(b, L.flux, L.flux_len);
    B.partial = reinterpret_cast<double *>(b + L.partial);
    return B;
}



int launch_prims(const Geom &g, const StateP &st, const Prims &P, uint32_t *status,
                 hipStream_t s)
{
    Observe o(VLCT_KERNEL_PRIMS, s);
    k_prims<<<xcd_grid(nblk_prims(g)), kBlock, 0, s>>>(g, st, P, status);
    return hipGetLastError() == hipSuccess ? VLCT_OK : VLCT_EHIP;
}

// face fluxes of a stage from its primitives P (and its stored face fields)
int launch_fluxes(const Geom &g, const StateP &st, const Prims &P, const Flux &F, int recon,
                  uint32_t *status, hipStream_t s)
{
    if (recon == VLCT_RECON_PCM) {
        // one thread per face
#define VLCT_FLUX(D)                                                                      \
    {                                                                                     \
        Observe o(VLCT_KERNEL_FLUX_PCM, s);                                               \
        k_flux<D, VLCT_RECON_PCM><<<xcd_grid(nblk_flux(g, D)), kBlock, 0, s>>>(g, st, P, F, status); \
    }
        VLCT_FLUX(0) VLCT_FLUX(1) VLCT_FLUX(2)
#undef VLCT_FLUX
    } else {
        // one reconstruction per cell and axis, x by rows, y and z by column marches
        const int kid = VLCT_KERNEL_FLUX_RECON;
#define VLCT_RECON3(R)                                                                        \
    {                                                                                         \
        { Observe o(kid, s); k_flux_recon_x<R><<<xcd_grid(nblk_row(g)), kBlock, 0, s>>>(g, st, P, F, status); } \
        { Observe o(kid, s);                                                                  \
          if (march_segment(g, 1) == 8)                                                        \
              k_flux_recon_march<1, R, 8><<<xcd_grid(nblk_march(g, 1, 8)), kBlock, 0, s>>>(g, st, P, F, status); \
          else                                                                                 \
              k_flux_recon_march<1, R><<<xcd_grid(nblk_march(g, 1)), kBlock, 0, s>>>(g, st, P, F, status); } \
        { Observe o(kid, s);                                                                  \
          if (march_segment(g, 2) == 8)                                                        \
              k_flux_recon_march<2, R, 8><<<xcd_grid(nblk_march(g, 2, 8)), kBlock, 0, s>>>(g, st, P, F, status); \
          else                                                                                 \
              k_flux_recon_march<2, R><<<xcd_grid(nblk_march(g, 2)), kBlock, 0, s>>>(g, st, P, F, status); } \
    }
        switch (recon) {
        case VLCT_RECON_PLMC: VLCT_RECON3(VLCT_RECON_PLMC) break;
        case VLCT_RECON_PPMC: VLCT_RECON3(VLCT_RECON_PPMC) break;
        case VLCT_RECON_PLMP: VLCT_RECON3(VLCT_RECON_PLMP) break;
        default: VLCT_RECON3(VLCT_RECON_PPMP) break;
        }
#undef VLCT_RECON3
    }
    return hipGetLastError() == hipSuccess ? VLCT_OK : VLCT_EHIP;
}

// CT edge fields + update: full = false is the half step into `out` (Steps
// 4-5), full = true the full step from `base` (Steps 8-9)
int launch_ct(const Geom &g, bool full, const Prims &P, const Flux &F, const StateP &base,
              const StateW &out, const double *dt_dev, uint32_t *status, hipStream_t s)
{
    Observe o(full ? VLCT_KERNEL_UPDATE_FULL : VLCT_KERNEL_UPDATE_HALF, s);
    if (full)
        k_ct_update<true><<<xcd_grid(nblk_ct(g)), kCt, 0, s>>>(g, P, F, base, out, dt_dev, status,
                                                               nullptr);
    else
        k_ct_update<false><<<xcd_grid(nblk_ct(g)), kCt, 0, s>>>(g, P, F, base, out, dt_dev,
                                                                status, nullptr);
    return hipGetLastError() == hipSuccess ? VLCT_OK : VLCT_EHIP;
}

// the whole predictor (Steps 2-5) in one kernel: U^n -> U^{n+1/2}; with
// `side` (3 arrays, tape layout) it also records the faces' upwind sides
static int launch_pred(const Geom &g, const StateP &st, const StateW &half, const Prims &P,
                       const double *dt_dev, uint32_t *status, uint8_t *const *side,
                       hipStream_t s)
{
    {
        Observe o(VLCT_KERNEL_PREDICTOR, s);
        uint8_t *s0 = side ? side[0] : nullptr, *s1 = side ? side[1] : nullptr,
                *s2 = side ? side[2] : nullptr;
        if (g.pred_chunk == 0)
            k_pred<true><<<xcd_grid(nblk_pred(g)), kPredThreads, 0, s>>>(g, st, half, P, dt_dev,
                                                                        status, s0, s1, s2);
        else
            k_pred<false><<<xcd_grid(nblk_pred(g)), kPredThreads, 0, s>>>(g, st, half, P, dt_dev,
                                                                         status, s0, s1, s2);
    }
    // ghost layers of the half-step primitives
    Observe o(VLCT_KERNEL_PRIMS, s);
    k_prims_ghost<<<xcd_grid((ghost_cells(g) + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        g, as_const(half), P, status);
    return hipGetLastError() == hipSuccess ? VLCT_OK : VLCT_EHIP;
}

// the full step's CT update with the CFL reduction of the new state fused in
// (one partial per CT block), then the final reduction into dt_out
static int launch_ct_dt(const Geom &g, const Prims &P, const Flux &F, const StateP &base,
                        const StateW &out, const double *dt_dev, uint32_t *status,
                        double *partial, double *dt_out, hipStream_t s)
{
    {
        Observe o(VLCT_KERNEL_UPDATE_FULL, s);
        k_ct_update<true, true><<<xcd_grid(nblk_ct(g)), kCt, 0, s>>>(g, P, F, base, out, dt_dev,
                                                                     status, partial);
    }
    Observe o(VLCT_KERNEL_DT_FINAL, s);
    k_dt_final<<<1, 1024, 0, s>>>(partial, (int)nblk_ct(g), g.cfl, dt_out);
    return hipGetLastError() == hipSuccess ? VLCT_OK : VLCT_EHIP;
}

__global__ void k_pack_sides(Geom g, Flux F, uint8_t *s0, uint8_t *s1, uint8_t *s2)
{
    const idx_t N = (idx_t)g.n[0] * g.n[1] * g.n[2];
    const idx_t t = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const int i = (int)(t % g.n[0]), j = (int)((t / g.n[0]) % g.n[1]),
              k = (int)(t / ((idx_t)g.n[0] * g.n[1]));
    s0[t] = side_code(F.sg[0][fidx(g, 0, i, j, k)]);
    s1[t] = side_code(F.sg[1][fidx(g, 1, i, j, k)]);
    s2[t] = side_code(F.sg[2][fidx(g, 2, i, j, k)]);
}

int launch_pack_sides(const Geom &g, const Flux &F, uint8_t *const side[3], hipStream_t s)
{
    const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    k_pack_sides<<<nblocks(N), kBlock, 0, s>>>(g, F, side[0], side[1], side[2]);
    return hipGetLastError() == hipSuccess ? VLCT_OK : VLCT_EHIP;
}

static int launch_dt(const Geom &g, const StateP &st, const Bound &B, const Layout &L,
                     double *dt_out, uint32_t *status, hipStream_t s)
{
    const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    Observe o(VLCT_KERNEL_DT, s);
    k_dt_partial<<<nblocks(N), kBlock, 0, s>>>(g, st, B.partial, status);
    k_dt_final<<<1, 1024, 0, s>>>(B.partial, (int)L.npartial, g.cfl, dt_out);
    return hipGetLastError() == hipSuccess ? VLCT_OK : VLCT_EHIP;
}

constexpr int kMaxBatch = 1 << 16;

// the instance table, then the clipped dt and active flag of every instance
// (used by vlct_step_batch_until)
static size_t batch_table_bytes(int count)
{
    return align_up((size_t)count * sizeof(Inst)) + align_up((size_t)count * sizeof(double)) +
           align_up((size_t)count * sizeof(int));
}
static double *batch_dt_eff(void *ws, int count)
{
    return reinterpret_cast<double *>(static_cast<char *>(ws) +
                                      align_up((size_t)count * sizeof(Inst)));
}
static int *batch_active(void *ws, int count)
{
    return reinterpret_cast<int *>(reinterpret_cast<char *>(batch_dt_eff(ws, count)) +
                                   align_up((size_t)count * sizeof(double)));
}

// instance records with workspace regions and flattened block offsets;
// returns the per-slot block totals through `total`
static void batch_records(int count, const vlct_grid *grids, const vlct_state *in,
                          const vlct_state *out, const double *dt_dev, double *next_dt_dev,
                          uint32_t *status_dev, const uint8_t *plan, void *ws,
                          std::vector<Inst> &rec, idx_t total[kSlots])
{
    rec.resize(count);
    size_t off = batch_table_bytes(count);
    for (int s = 0; s < kSlots; ++s) total[s] = 0;
    for (int i = 0; i < count; ++i) {
        const Geom g = make_geom(&grids[i]);
        const Layout L = layout(g);
        const Bound B = bind(L, static_cast<char *>(ws) + off);
        off += L.total;
        Inst &r = rec[i];
        r.g = g;
        r.in = as_const(&in[i]);
        r.out = as_mut(&out[i]);
        r.half = B.half;
        r.P = B.P;
        r.F = B.F;
        r.partial = B.partial;
        r.dt = dt_dev + i;
        r.next_dt = next_dt_dev ? next_dt_dev + i : nullptr;
        r.status = status_dev ? status_dev + i : nullptr;
        r.active = nullptr;
        r.t = nullptr;
        const int cv = plan ? (plan[i] & 15) : 0, mv = plan ? (plan[i] >> 4) : 0;
        idx_t nb[kSlots] = {};
        nb[kSlotPred] = nblk_pred_shares(g);
        nb[kSlotGhost] = (ghost_cells(g) + kBlock - 1) / kBlock;
        nb[kSlotPrims] = nblk_prims(g);
        for (int d = 0; d < 3; ++d) nb[kSlotFlux0 + d] = nblk_flux(g, d);
        nb[kSlotRow] = nblk_row(g);
        nb[kSlotMarch1 + mv] = nblk_march(g, 1, march_len(mv));
        nb[kSlotMarch2 + mv] = nblk_march(g, 2, march_len(mv));
        nb[kSlotCt + cv] = nblk_ct(g, ct_tx(cv), ct_ty(cv));
        nb[kSlotDt] = nblk_dt(g);
        for (int s = 0; s < kSlots; ++s) {
            r.start[s] = total[s];
            total[s] += nb[s];
        }
    }
}

// every output array belongs to one instance, and an input array is shared
// only with the same field of its own instance's output (in-place)
static bool batch_aliasing_ok(int count, const vlct_state *in, const vlct_state *out)
{
    std::unordered_map<const void *, long> owner;  // pointer -> instance * 8 + field
    auto fields = [](const vlct_state &st, int f) -> const void * {
        const double *p[8] = {st.rho, st.mx, st.my, st.mz, st.E, st.bx, st.by, st.bz};
        return p[f];
    };
    for (int i = 0; i < count; ++i)
        for (int f = 0; f < 8; ++f)
            if (!owner.emplace(fields(out[i], f), (long)i * 8 + f).second) return false;
    for (int i = 0; i < count; ++i)
        for (int f = 0; f < 8; ++f) {
            auto it = owner.find(fields(in[i], f));
            if (it != owner.end() && it->second != (long)i * 8 + f) return false;
        }
    // an instance is either fully in place or fully out of place
    for (int i = 0; i < count; ++i) {
        int same = 0;
        for (int f = 0; f < 8; ++f) same += fields(in[i], f) == fields(out[i], f);
        if (same != 0 && same != 8) return false;
    }
    return true;
}

// ---------------------------------------------------------------------------
// static scratch of vlct_step_noalloc: the workspace of vlct_step in a
// file-scope device array, so a caller that cannot allocate device memory can
// still step a grid whose workspace fits.  Each device holds its own copy; its
// address comes from hipGetSymbolAddress once per device (the array's name in
// host code is a host-side stand-in, never a device address).  Nothing in the
// step's workspace has to start at zero: every kernel writes what a later one
// reads within the same call.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = VLCT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kScratchDevices = 64;
static std::atomic<void *> g_scratch_addr[kScratchDevices];
static std::mutex g_scratch_mutex;

// device address of the current device's scratch array
static int scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return VLCT_EHIP;
    void *p = g_scratch_addr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        p = g_scratch_addr[dev].load(std::memory_order_relaxed);
        if (!p) {
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return VLCT_EHIP;
            g_scratch_addr[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return VLCT_OK;
}

// `out` must be `in` itself (all eight arrays the same) or use memory that no
// input array overlaps, and no two output arrays may overlap: compared as
// address ranges [p, p + bytes) of the grid's field sizes
static bool in_out_ok(const vlct_grid *vg, const vlct_state *in, const vlct_state *out,
                      bool &all_same)
{
    const int n[3] = {vg->nx, vg->ny, vg->nz};
    const double *pi[8] = {in->rho, in->mx, in->my, in->mz, in->E, in->bx, in->by, in->bz};
    const double *po[8] = {out->rho, out->mx, out->my, out->mz, out->E, out->bx, out->by, out->bz};
    auto overlap = [&](const double *a, int fa, const double *b, int fb) {
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
        const uintptr_t a1 = a0 + field_len(n, fa) * sizeof(double);
        const uintptr_t b1 = b0 + field_len(n, fb) * sizeof(double);
        return a0 < b1 && b0 < a1;
    };
    all_same = true;
    for (int f = 0; f < 8; ++f) all_same &= pi[f] == po[f];
    for (int f = 0; f < 8; ++f)
        for (int h = f + 1; h < 8; ++h)
            if (overlap(po[f], f, po[h], h)) return false;
    if (all_same) return true;
    for (int f = 0; f < 8; ++f)
        for (int h = 0; h < 8; ++h)
            if (overlap(po[f], f, pi[h], h)) return false;
    return true;
}

}  // namespace vlct

using namespace vlct;

extern "C" {

size_t vlct_workspace_bytes(const vlct_grid *g)
{
    if (!grid_ok(g)) return 0;
    return layout(make_geom(g)).total;
}

int vlct_cfl_dt(const vlct_grid *vg, const vlct_state *s, double *dt_dev, void *ws,
                size_t ws_bytes, void *stream)
{
    if (!grid_ok(vg) || !state_ok(s) || !dt_dev) return VLCT_EINVAL;
    const Geom g = make_geom(vg);
    const Layout L = layout(g);
    if (!ws || ws_bytes < L.total) return VLCT_EWORKSPACE;
    const Bound B = bind(L, ws);
    return launch_dt(g, as_const(s), B, L, dt_dev, nullptr, static_cast<hipStream_t>(stream));
}

int vlct_step(const vlct_grid *vg, const vlct_state *in, const vlct_state *out,
              const double *dt_dev, double *next_dt_dev, uint32_t *status_dev, void *ws,
              size_t ws_bytes, void *stream)
{
    if (!grid_ok(vg) || !state_ok(in) || !state_ok(out) || !dt_dev) return VLCT_EINVAL;
    bool all_same = false;
    if (!in_out_ok(vg, in, out, all_same)) return VLCT_EINVAL;
    const Geom g = make_geom(vg);
    const Layout L = layout(g);
    if (!ws || ws_bytes < L.total) return VLCT_EWORKSPACE;
    const Bound B = bind(L, ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const StateP sin = as_const(in);
    // predictor (Steps 2-5)
    int rc = launch_pred(g, sin, B.half, B.P, dt_dev, status_dev, nullptr, s);
    // corrector (Steps 6-9) on the half-step primitives the predictor left in B.P
    const StateP half = as_const(B.half);
    if (!rc) rc = launch_fluxes(g, half, B.P, B.F, vg->recon, status_dev, s);
    if (rc) return rc;
    // the CFL reduction rides on the full update unless the step is in place
    // (it reads the base field on faces that other threads update)
    if (next_dt_dev && !all_same)
        return launch_ct_dt(g, B.P, B.F, sin, as_mut(out), dt_dev, status_dev, B.partial,
                            next_dt_dev, s);
    rc = launch_ct(g, true, B.P, B.F, sin, as_mut(out), dt_dev, status_dev, s);
    if (rc) return rc;
    if (next_dt_dev) return launch_dt(g, as_const(out), B, L, next_dt_dev, status_dev, s);
    return VLCT_OK;
}

int vlct_step_noalloc(const vlct_grid *vg, const vlct_state *in, const vlct_state *out,
                      const double *dt_dev, double *next_dt_dev, uint32_t *status_dev,
                      void *stream)
{
    if (!grid_ok(vg) || !state_ok(in) || !state_ok(out) || !dt_dev) return VLCT_EINVAL;
    if (layout(make_geom(vg)).total > kScratchBytes) return VLCT_ESCRATCH;
    void *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc) return rc;
    return vlct_step(vg, in, out, dt_dev, next_dt_dev, status_dev, ws, kScratchBytes, stream);
}

size_t vlct_tape_bytes(const vlct_grid *g)
{
    if (!grid_ok(g)) return 0;
    const int n[3] = {g->nx, g->ny, g->nz};
    return tape_layout(n).total;
}

int vlct_step_taped(const vlct_grid *vg, const vlct_state *in, const vlct_state *out,
                    const double *dt_dev, double *next_dt_dev, uint32_t *status_dev, void *ws,
                    size_t ws_bytes, void *tape, size_t tape_bytes, void *stream)
{
    if (!grid_ok(vg) || !state_ok(in) || !state_ok(out) || !dt_dev) return VLCT_EINVAL;
    bool all_same = false;
    if (!in_out_ok(vg, in, out, all_same)) return VLCT_EINVAL;
    const Geom g = make_geom(vg);
    const Layout L = layout(g);
    const TapeLayout T = tape_layout(g.n);
    if (!ws || ws_bytes < L.total || !tape || tape_bytes < T.total) return VLCT_EWORKSPACE;
    const Bound B = bind(L, ws);
    char *tb = static_cast<char *>(tape);
    StateW half;
    for (int f = 0; f < 8; ++f) {
        double *a = reinterpret_cast<double *>(tb + T.half[f]);
        if (f < 5) half.u[f] = a; else half.b[f - 5] = a;
    }
    uint8_t *side[2][3];
    for (int h = 0; h < 2; ++h)
        for (int d = 0; d < 3; ++d) side[h][d] = reinterpret_cast<uint8_t *>(tb + T.side[h][d]);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const StateP sin = as_const(in);
    // the steps of vlct_step with the half-step state and both stages' upwind
    // sides kept in the tape
    int rc = launch_pred(g, sin, half, B.P, dt_dev, status_dev, side[0], s);
    const StateP hc = as_const(half);
    if (!rc) rc = launch_fluxes(g, hc, B.P, B.F, vg->recon, status_dev, s);
    if (!rc) rc = launch_pack_sides(g, B.F, side[1], s);
    if (rc) return rc;
    // the CFL reduction rides on the full update unless the step is in place
    // (it reads the base field on faces that other threads update)
    if (next_dt_dev && !all_same)
        return launch_ct_dt(g, B.P, B.F, sin, as_mut(out), dt_dev, status_dev, B.partial,
                            next_dt_dev, s);
    rc = launch_ct(g, true, B.P, B.F, sin, as_mut(out), dt_dev, status_dev, s);
    if (rc) return rc;
    if (next_dt_dev) return launch_dt(g, as_const(out), B, L, next_dt_dev, status_dev, s);
    return VLCT_OK;
}

const char *vlct_strerror(int code)
{
    switch (code) {
    case VLCT_OK: return "ok";
    case VLCT_EINVAL: return "invalid argument (grid descriptor, state pointers or dt)";
    case VLCT_EWORKSPACE: return "workspace missing or smaller than vlct_workspace_bytes()";
    case VLCT_EHIP: return "HIP launch or runtime error";
    case VLCT_EUNSUPPORTED: return "unsupported option";
    case VLCT_ESCRATCH:
        return "grid needs more workspace than the static scratch of vlct_step_noalloc "
               "(VLCT_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown error code";
    }
}

int vlct_abi_version(void) { return VLCT_ABI_VERSION; }

int vlct_step_observed(const vlct_grid *g, const vlct_state *in, const vlct_state *out,
                       const double *dt_dev, double *next_dt_dev, uint32_t *status_dev, void *ws,
                       size_t ws_bytes, void *stream, vlct_launch_observer cb, void *user)
{
    if (!cb) return VLCT_EINVAL;
    const ObserverCtx ctx{cb, user};
    struct Scope {
        explicit Scope(const ObserverCtx *c) { t_observer = c; }
        ~Scope() { t_observer = nullptr; }
    } scope(&ctx);
    return vlct_step(g, in, out, dt_dev, next_dt_dev, status_dev, ws, ws_bytes, stream);
}

size_t vlct_batch_workspace_bytes(const vlct_grid *grids, int count)
{
    if (!grids || count < 1 || count > kMaxBatch) return 0;
    size_t tot = batch_table_bytes(count);
    for (int i = 0; i < count; ++i) {
        if (!grid_ok(&grids[i])) return 0;
        tot += layout(make_geom(&grids[i])).total;
    }
    return tot;
}

int vlct_step_batch(int count, const vlct_grid *grids, const vlct_state *in,
                    const vlct_state *out, const double *dt_dev, double *next_dt_dev,
                    uint32_t *status_dev, void *ws, size_t ws_bytes, void *stream)
{
    return vlct_step_batch_plan(count, grids, in, out, dt_dev, next_dt_dev, status_dev, nullptr,
                                ws, ws_bytes, stream);
}

static int batch_args(int count, const vlct_grid *grids, const vlct_state *in,
                      const vlct_state *out, const double *dt_dev, const uint8_t *plan)
{
    if (count < 1 || count > kMaxBatch || !grids || !in || !out || !dt_dev) return VLCT_EINVAL;
    for (int i = 0; i < count; ++i)
        if (!grid_ok(&grids[i]) || !state_ok(&in[i]) || !state_ok(&out[i])) return VLCT_EINVAL;
    if (plan)
        for (int i = 0; i < count; ++i)
            if ((plan[i] & 15) >= kCtVariants || (plan[i] >> 4) >= kMarchVariants) return VLCT_EINVAL;
    for (int i = 1; i < count; ++i)
        if (grids[i].recon != grids[0].recon) return VLCT_EUNSUPPORTED;
    if (!batch_aliasing_ok(count, in, out)) return VLCT_EINVAL;
    return VLCT_OK;
}

// the batched step; with t_dev / t_end_dev (device, count each) every
// instance runs only while t < t_end, by min(dt, t_end - t), and advances t
static int batch_step(int count, const vlct_grid *grids, const vlct_state *in,
                      const vlct_state *out, const double *dt_dev, double *next_dt_dev,
                      uint32_t *status_dev, const uint8_t *plan, void *ws, size_t ws_bytes,
                      void *stream, double *t_dev, const double *t_end_dev)
{
    const int arc = batch_args(count, grids, in, out, dt_dev, plan);
    if (arc) return arc;
    const size_t need = vlct_batch_workspace_bytes(grids, count);
    if (!ws || ws_bytes < need) return VLCT_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<Inst> rec;
    idx_t tot[kSlots];
    batch_records(count, grids, in, out, dt_dev, next_dt_dev, status_dev, plan, ws, rec, tot);
    if (t_dev) {
        double *dt_eff = batch_dt_eff(ws, count);
        int *active = batch_active(ws, count);
        kb_clip<<<(count + 255) / 256, 256, 0, s>>>(count, dt_dev, t_dev, t_end_dev, dt_eff,
                                                    active);
        for (int i = 0; i < count; ++i) {
            rec[i].dt = dt_eff + i;
            rec[i].active = active + i;
            rec[i].t = t_dev + i;
        }
    }
    Inst *tab = static_cast<Inst *>(ws);
    for (int first = 0; first < count; first += kPackChunk) {
        PackArgs a;
        a.tab = tab;
        a.first = first;
        a.n = std::min(kPackChunk, count - first);
        for (int q = 0; q < a.n; ++q) a.rec[q] = rec[first + q];
        k_pack<<<1, 64, 0, s>>>(a);
    }
    const int recon = grids[0].recon;
    // predictor (Steps 2-5)
    {
        Observe o(VLCT_KERNEL_PREDICTOR, s);
        kb_pred<<<xcd_grid(tot[kSlotPred]), kPredThreads, 0, s>>>(tab, count, tot[kSlotPred]);
    }
    {
        Observe o(VLCT_KERNEL_PRIMS, s);
        kb_prims_ghost<<<xcd_grid(tot[kSlotGhost]), kBlock, 0, s>>>(tab, count, tot[kSlotGhost]);
    }
#define VLCT_BCT(FULL, V)                                                                 \
    if (tot[kSlotCt + V]) {                                                                   \
        Observe o(FULL ? VLCT_KERNEL_UPDATE_FULL : VLCT_KERNEL_UPDATE_HALF, s);                \
        kb_ct<FULL, V><<<xcd_grid(tot[kSlotCt + V]), kCt, 0, s>>>(tab, count, tot[kSlotCt + V]); \
    }
    // corrector (Steps 6-9); the predictor wrote the interior primitives
#define VLCT_BMARCH(D, R, V)                                                                  \
    if (tot[(D == 1 ? kSlotMarch1 : kSlotMarch2) + V]) {                                      \
        const idx_t n = tot[(D == 1 ? kSlotMarch1 : kSlotMarch2) + V];                        \
        Observe o(VLCT_KERNEL_FLUX_RECON, s);                                                 \
        kb_march<D, R, V><<<xcd_grid(n), kBlock, 0, s>>>(tab, count, n);                      \
    }
#define VLCT_BRECON(R)                                                                        \
    {                                                                                         \
        { Observe o(VLCT_KERNEL_FLUX_RECON, s);                                                \
          kb_recon_x<R><<<xcd_grid(tot[kSlotRow]), kBlock, 0, s>>>(tab, count, tot[kSlotRow]); } \
        VLCT_BMARCH(1, R, 0) VLCT_BMARCH(1, R, 1) VLCT_BMARCH(1, R, 2)                        \
        VLCT_BMARCH(2, R, 0) VLCT_BMARCH(2, R, 1) VLCT_BMARCH(2, R, 2)                        \
    }
    switch (recon) {
    case VLCT_RECON_PCM:
        for (int d = 0; d < 3; ++d) {
            Observe o(VLCT_KERNEL_FLUX_PCM, s);
            const idx_t n = tot[kSlotFlux0 + d];
            if (d == 0) kb_flux_pcm<0><<<xcd_grid(n), kBlock, 0, s>>>(tab, count, n, 1);
            if (d == 1) kb_flux_pcm<1><<<xcd_grid(n), kBlock, 0, s>>>(tab, count, n, 1);
            if (d == 2) kb_flux_pcm<2><<<xcd_grid(n), kBlock, 0, s>>>(tab, count, n, 1);
        }
        break;
    case VLCT_RECON_PLMC: VLCT_BRECON(VLCT_RECON_PLMC) break;
    case VLCT_RECON_PPMC: VLCT_BRECON(VLCT_RECON_PPMC) break;
    case VLCT_RECON_PLMP: VLCT_BRECON(VLCT_RECON_PLMP) break;
    default: VLCT_BRECON(VLCT_RECON_PPMP) break;
    }
#undef VLCT_BRECON
#undef VLCT_BMARCH
    VLCT_BCT(true, 0) VLCT_BCT(true, 1) VLCT_BCT(true, 2)
#undef VLCT_BCT
    if (next_dt_dev) {
        Observe o(VLCT_KERNEL_DT, s);
        kb_dt_partial<<<(unsigned)tot[kSlotDt], kBlock, 0, s>>>(tab, count, tot[kSlotDt]);
        kb_dt_final<<<count, 1024, 0, s>>>(tab);
    }
    return hipGetLastError() == hipSuccess ? VLCT_OK : VLCT_EHIP;
}

int vlct_step_batch_plan(int count, const vlct_grid *grids, const vlct_state *in,
                         const vlct_state *out, const double *dt_dev, double *next_dt_dev,
                         uint32_t *status_dev, const uint8_t *plan, void *ws, size_t ws_bytes,
                         void *stream)
{
    return batch_step(count, grids, in, out, dt_dev, next_dt_dev, status_dev, plan, ws, ws_bytes,
                      stream, nullptr, nullptr);
}

int vlct_step_batch_until(int count, const vlct_grid *grids, const vlct_state *states,
                          const double *dt_dev, double *next_dt_dev, uint32_t *status_dev,
                          double *t_dev, const double *t_end_dev, const uint8_t *plan, void *ws,
                          size_t ws_bytes, void *stream)
{
    if (!t_dev || !t_end_dev || !next_dt_dev) return VLCT_EINVAL;
    return batch_step(count, grids, states, states, dt_dev, next_dt_dev, status_dev, plan, ws,
                      ws_bytes, stream, t_dev, t_end_dev);
}

int vlct_batch_tune(int count, const vlct_grid *grids, const vlct_state *in,
                    const vlct_state *out, const double *dt_dev, void *ws, size_t ws_bytes,
                    void *stream, int reps, uint8_t *plan)
{
    const int arc = batch_args(count, grids, in, out, dt_dev, nullptr);
    if (arc) return arc;
    if (!plan || reps < 1 || reps > 100) return VLCT_EINVAL;
    // the trial steps write `out` and leave `in` unchanged
    for (int i = 0; i < count; ++i)
        if (in[i].rho == out[i].rho) return VLCT_EINVAL;
    if (!ws || ws_bytes < vlct_batch_workspace_bytes(grids, count)) return VLCT_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return VLCT_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return VLCT_EHIP;
    }
    // mean time of one batched step under plan p (one untimed step first)
    auto time_plan = [&](const std::vector<uint8_t> &p, float &ms) -> int {
        int rc = vlct_step_batch_plan(count, grids, in, out, dt_dev, nullptr, nullptr, p.data(),
                                      ws, ws_bytes, stream);
        if (rc) return rc;
        if (hipEventRecord(e0, s) != hipSuccess) return VLCT_EHIP;
        for (int r = 0; r < reps && !rc; ++r)
            rc = vlct_step_batch_plan(count, grids, in, out, dt_dev, nullptr, nullptr, p.data(),
                                      ws, ws_bytes, stream);
        if (rc) return rc;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return VLCT_EHIP;
        ms /= (float)reps;
        return VLCT_OK;
    };
    // size classes by the x extent (the CT tile's long side): <= 24, <= 48, <= 96, larger;
    // each class's CT tile, then its march segment, is changed while the rest
    // of the batch keeps its current choice, and kept if the whole batched step
    // gets at least 1% faster
    std::vector<int> cls(count);
    for (int i = 0; i < count; ++i) {
        const int nx = grids[i].nx;
        cls[i] = nx <= 24 ? 0 : (nx <= 48 ? 1 : (nx <= 96 ? 2 : 3));
    }
    std::vector<uint8_t> cur(count, 0);
    float best = 0.0f;
    int rc = time_plan(cur, best);
    for (int c = 0; c < 4 && !rc; ++c) {
        bool present = false;
        for (int i = 0; i < count; ++i) present |= cls[i] == c;
        if (!present) continue;
        for (int field = 0; field < 2 && !rc; ++field) {
            const int nv = field == 0 ? kCtVariants : kMarchVariants;
            for (int v = 0; v < nv && !rc; ++v) {
                std::vector<uint8_t> trial = cur;
                bool changed = false;
                for (int i = 0; i < count; ++i) {
                    if (cls[i] != c) continue;
                    const uint8_t b = field == 0 ? (uint8_t)((trial[i] & 0xF0) | v)
                                                 : (uint8_t)((trial[i] & 0x0F) | (v << 4));
                    changed |= b != trial[i];
                    trial[i] = b;
                }
                if (!changed) continue;
                float ms = 0.0f;
                rc = time_plan(trial, ms);
                if (!rc && ms < 0.99f * best) {
                    best = ms;
                    cur = trial;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    for (int i = 0; i < count; ++i) plan[i] = cur[i];
    return VLCT_OK;
}

const char *vlct_kernel_name(int kernel)
{
    static const char *names[VLCT_KERNEL_COUNT] = {"prims",       "flux_pcm_hlld",
                                                   "flux_recon_hlld", "edges",
                                                   "update_half", "update_full",
                                                   "dt",          "dt_final",
                                                   "predictor"};
    return kernel >= 0 && kernel < VLCT_KERNEL_COUNT ? names[kernel] : "?";
}

}  // extern "C"
