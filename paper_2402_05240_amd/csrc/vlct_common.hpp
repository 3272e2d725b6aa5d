// vlct_common.hpp -- definitions shared by the step kernels (vlct.hip) and
// the adjoint kernels (vlct_adjoint.hip): launch geometry, index maps of the
// state and workspace arrays, state views and argument checks.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <cstring>

#include "../../include/vlct.h"

namespace vlct {

constexpr int kGhost = 3;          // ghost layers of the primitive workspace
constexpr int kBlock = 256;        // threads per block (4 wave64s)
constexpr int kMaxN = 4096;

using idx_t = long long;

// MI355X dispatches consecutive workgroups round-robin to its 8 XCDs, each with
// its own L2.  Kernels launched on xcd_grid(n) blocks read their logical block
// from xcd_block(n): hardware block b works on logical block
// (b mod 8) * ceil(n/8) + b / 8, so every XCD sweeps one contiguous slab of
// the domain and neighbouring rows and planes meet in the same L2.
constexpr int kXcd = 8;
__host__ __device__ __forceinline__ idx_t xcd_per(idx_t n) { return (n + kXcd - 1) / kXcd; }
__device__ __forceinline__ idx_t xcd_block(idx_t n)
{
    const idx_t b = blockIdx.x;
    return (b % kXcd) * xcd_per(n) + b / kXcd;
}

// ---------------------------------------------------------------------------
// geometry shared by every kernel
// ---------------------------------------------------------------------------
struct Geom {
    int n[3];
    int bc[3];
    double dl[3];
    double gamma, gm1i, cfl;
    int p[3];  // padded primitive dims n + 2G
    int ct_planes;    // z planes a CT block marches through
    int pred_slab;    // z planes per slab of the fused predictor's pair order
    int pred_chunk;   // (column tile, plane) pairs of one fused predictor block
                      // (0: one (slab, tile) per block)
};

__host__ __device__ __forceinline__ int map_cell(int i, int n, int bc)
{
    if (bc == VLCT_BC_PERIODIC) {
        // one period either side without an integer division
        if (i >= 0 && i < n) return i;
        if (i < 0 && i >= -n) return i + n;
        if (i >= n && i < 2 * n) return i - n;
        const int m = i % n;
        return m < 0 ? m + n : m;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}
// normal-face index: periodic faces wrap into [0, n-1], outflow clamps into [0, n]
__host__ __device__ __forceinline__ int map_face(int i, int n, int bc)
{
    if (bc == VLCT_BC_PERIODIC) return map_cell(i, n, bc);
    return i < 0 ? 0 : (i > n ? n : i);
}

// stored face arrays of the state: axis d has n_d + 1 faces along d
__device__ __forceinline__ idx_t face_store(const Geom &g, int d, int i, int j, int k)
{
    const idx_t nx = g.n[0] + (d == 0), ny = g.n[1] + (d == 1);
    return ((idx_t)k * ny + j) * nx + i;
}

__device__ __forceinline__ idx_t cell_store(const Geom &g, int i, int j, int k)
{
    return ((idx_t)k * g.n[1] + j) * g.n[0] + i;
}

// padded primitive index, i,j,k in [-G, n+G-1]
__device__ __forceinline__ idx_t pidx(const Geom &g, int i, int j, int k)
{
    return ((idx_t)(k + kGhost) * g.p[1] + (j + kGhost)) * g.p[0] + (i + kGhost);
}

// flux arrays of axis d: normal index in [0, n_d], transverse in [-1, n_e]
__host__ __device__ __forceinline__ idx_t flux_dim(const int n[3], int d, int e)
{
    return n[e] + (e == d ? 1 : 2);
}
__device__ __forceinline__ idx_t fidx(const Geom &g, int d, int i, int j, int k)
{
    const idx_t X = flux_dim(g.n, d, 0), Y = flux_dim(g.n, d, 1);
    return ((idx_t)(k + (d != 2)) * Y + (j + (d != 1))) * X + (i + (d != 0));
}

struct StateP {
    const double *u[5];
    const double *b[3];
};
struct StateW {
    double *u[5];
    double *b[3];
};
struct Prims {
    double *w[8];  // rho, vx, vy, vz, P, Bcx, Bcy, Bcz on padded cells
};
inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Flux {
    double *f[3][7];  // per axis: 7 sweep-frame flux components
    int8_t *sg[3];    // per axis: CT upwind indicator (+1, -1, 0), the sign of S_M
};

// bytes of one axis' flux arrays (7 doubles and the indicator per face)
inline size_t flux_axis_bytes(size_t len)
{
    return 7 * align_up(len * sizeof(double)) + align_up(len);
}

inline Flux bind_flux(char *base, const size_t off[3], const size_t len[3])
{
    Flux F;
    for (int d = 0; d < 3; ++d) {
        for (int c = 0; c < 7; ++c)
            F.f[d][c] = reinterpret_cast<double *>(base + off[d] + c * align_up(len[d] * sizeof(double)));
        F.sg[d] = reinterpret_cast<int8_t *>(base + off[d] + 7 * align_up(len[d] * sizeof(double)));
    }
    return F;
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
inline bool grid_ok(const vlct_grid *g)
{
    if (!g) return false;
    const int n[3] = {g->nx, g->ny, g->nz};
    for (int d = 0; d < 3; ++d) {
        if (n[d] < 1 || n[d] > kMaxN) return false;
        if (g->bc[d] != VLCT_BC_PERIODIC && g->bc[d] != VLCT_BC_OUTFLOW) return false;
    }
    if (!(g->dx > 0.0) || !(g->dy > 0.0) || !(g->dz > 0.0)) return false;
    if (!(g->gamma > 1.0) || !(g->cfl > 0.0 && g->cfl <= 0.5)) return false;
    if (g->recon < VLCT_RECON_PCM || g->recon > VLCT_RECON_PPMP) return false;
    return true;
}

// Tile override for tests and tuning: the environment variable VLCT_TILES,
// read at every call, holds comma-separated key=value pairs (ct=4|8|16|32|64 CT
// planes per block, march=8|16 faces per corrector march segment, pred=N
// (column tile, plane) pairs per fused predictor block in one shared slab,
// predslab=P slabs of P planes one per predictor block, admarch=8|16 cells per adjoint march
// segment) that replace the size-dependent choices.  Every choice computes the
// same per-cell and per-face arithmetic; the forward results are bitwise the
// same, the adjoint's equal to the summation order of its accumulations.
// Returns 0 when `key` is not set.
inline int tile_override(const char *key)
{
    const char *env = std::getenv("VLCT_TILES");
    if (!env) return 0;
    const size_t kl = std::strlen(key);
    for (const char *p = env; *p;) {
        if (std::strncmp(p, key, kl) == 0 && p[kl] == '=') return std::atoi(p + kl + 1);
        const char *c = std::strchr(p, ',');
        if (!c) break;
        p = c + 1;
    }
    return 0;
}

// fused predictor column tile: kPredTx x kPredTy cells, its threads also
// covering a one-cell ring (34 x 15 columns, 510 threads of 512); one block
// per CU (123 KB of LDS, 256 VGPRs: two waves per SIMD)
constexpr int kPredTx = 32, kPredTy = 13;
constexpr int kPredBlocksPerCU = 1;
constexpr int kPredWavesPerSimd = 2;
constexpr int kNumCUs = 256;  // gfx950 (MI355X)

__host__ __device__ __forceinline__ long long pred_tiles(const Geom &g)
{
    const int ntx = (g.n[0] + (g.bc[0] == VLCT_BC_OUTFLOW) + kPredTx - 1) / kPredTx;
    const int nty = (g.n[1] + (g.bc[1] == VLCT_BC_OUTFLOW) + kPredTy - 1) / kPredTy;
    return (long long)ntx * nty;
}

inline Geom make_geom(const vlct_grid *vg)
{
    Geom g;
    g.n[0] = vg->nx;
    g.n[1] = vg->ny;
    g.n[2] = vg->nz;
    for (int d = 0; d < 3; ++d) {
        g.bc[d] = vg->bc[d];
        g.p[d] = g.n[d] + 2 * kGhost;
    }
    g.dl[0] = vg->dx;
    g.dl[1] = vg->dy;
    g.dl[2] = vg->dz;
    g.gamma = vg->gamma;
    g.gm1i = 1.0 / (vg->gamma - 1.0);
    g.cfl = vg->cfl;
    // CT blocks march 32 planes through a column tile of 64 x 8, halved down to
    // 8 while the grid has fewer than 1024 such blocks (4 per CU); one with
    // fewer than 256 blocks of 8 planes takes 4 (measured at 64^3 .. 256^3: 32
    // planes from 256^3 up, 8 at 128^3 and 192^3, 4 at 64^3)
    const long long cols = (long long)((g.n[0] + (g.bc[0] == VLCT_BC_OUTFLOW) + 63) / 64) *
                           ((g.n[1] + (g.bc[1] == VLCT_BC_OUTFLOW) + 7) / 8);
    g.ct_planes = 32;
    while (g.ct_planes > 8 && cols * ((g.n[2] + g.ct_planes - 1) / g.ct_planes) < 1024)
        g.ct_planes /= 2;
    if (g.ct_planes == 8 && cols * ((g.n[2] + 7) / 8) < 256) g.ct_planes = 4;
    // fused predictor (a run of p planes also solves the faces of one plane
    // beyond each end): either one (z slab of p planes, column tile) per block,
    // neighbouring tiles of a slab in neighbouring blocks so that they share
    // their ring columns in L2, p minimising (waves of resident blocks) x
    // (p + 2); or, where that leaves much of the last wave idle, the grid as
    // one slab shared out evenly over one wave, at least 4 planes a block
    // (measured: slabs at 64^3 and 256^3, one shared slab at 128^3)
    const long long tiles = pred_tiles(g), resident = (long long)kNumCUs * kPredBlocksPerCU;
    double best = -1.0;
    for (int p = 64; p >= 4; p /= 2) {
        const long long blocks = tiles * ((g.n[2] + p - 1) / p);
        const double cost = (double)((blocks + resident - 1) / resident) * (p + 2);
        if (best < 0.0 || cost < best) {
            best = cost;
            g.pred_slab = p;
            g.pred_chunk = 0;  // one (slab, tile) per block
        }
    }
    long long chunk = (tiles * g.n[2] + resident - 1) / resident;
    if (chunk < 4) chunk = 4;
    const double shared = (double)chunk + 2.0 * (1.0 + (double)chunk / g.n[2]);
    if (shared < 0.9 * best) {
        g.pred_slab = g.n[2];
        g.pred_chunk = (int)chunk;
    }
    const int oct = tile_override("ct"), opred = tile_override("pred");
    if (oct == 4 || oct == 8 || oct == 16 || oct == 32 || oct == 64) g.ct_planes = oct;
    const int oslab = tile_override("predslab");
    if (opred >= 1) {  // one shared slab, opred pairs per block
        g.pred_slab = g.n[2];
        g.pred_chunk = opred;
    }
    if (oslab >= 1) {  // slabs of oslab planes, one (slab, tile) per block
        g.pred_slab = oslab;
        g.pred_chunk = 0;
    }
    return g;
}

inline size_t field_len(const int n[3], int f)
{
    size_t nx = n[0], ny = n[1], nz = n[2];
    if (f < 5) return nx * ny * nz;
    if (f == 5) return (nx + 1) * ny * nz;
    if (f == 6) return nx * (ny + 1) * nz;
    return nx * ny * (nz + 1);
}

inline bool state_ok(const vlct_state *s)
{
    if (!s) return false;
    const double *p[8] = {s->rho, s->mx, s->my, s->mz, s->E, s->bx, s->by, s->bz};
    for (int f = 0; f < 8; ++f)
        if (!p[f]) return false;
    return true;
}

inline StateP as_const(const vlct_state *s)
{
    StateP p;
    p.u[0] = s->rho; p.u[1] = s->mx; p.u[2] = s->my; p.u[3] = s->mz; p.u[4] = s->E;
    p.b[0] = s->bx; p.b[1] = s->by; p.b[2] = s->bz;
    return p;
}

inline StateP as_const(const StateW &s)
{
    StateP p;
    for (int f = 0; f < 5; ++f) p.u[f] = s.u[f];
    for (int d = 0; d < 3; ++d) p.b[d] = s.b[d];
    return p;
}

inline StateW as_mut(const vlct_state *s)
{
    StateW p;
    p.u[0] = s->rho; p.u[1] = s->mx; p.u[2] = s->my; p.u[3] = s->mz; p.u[4] = s->E;
    p.b[0] = s->bx; p.b[1] = s->by; p.b[2] = s->bz;
    return p;
}


inline unsigned nblocks(size_t work) { return (unsigned)((work + kBlock - 1) / kBlock); }

// grid size (multiple of the XCD count) for a kernel that remaps with xcd_block
inline unsigned xcd_grid(size_t logical_blocks) { return (unsigned)(kXcd * xcd_per(logical_blocks)); }

// upwind side of a face from its CT indicator (the sign of S_M, Eq. emf-upwind):
// 0 for S_M > 0, 1 for S_M < 0, 2 for neither
__device__ __forceinline__ uint8_t side_code(double s)
{
    return s > 0.0 ? (uint8_t)0 : (s < 0.0 ? (uint8_t)1 : (uint8_t)2);
}

// tape of one step (vlct_step_taped): the half-step state and the upwind side
// of every interior face of both stages (one byte, at the index of the cell
// whose low face it is)
struct TapeLayout {
    size_t half[8], side[2][3], total;
};

inline TapeLayout tape_layout(const int n[3])
{
    TapeLayout T;
    size_t off = 0;
    for (int f = 0; f < 8; ++f) {
        T.half[f] = off;
        off += align_up(field_len(n, f) * sizeof(double));
    }
    const size_t N = (size_t)n[0] * n[1] * n[2];
    for (int h = 0; h < 2; ++h)
        for (int d = 0; d < 3; ++d) {
            T.side[h][d] = off;
            off += align_up(N);
        }
    T.total = off;
    return T;
}

// launches of the step kernels (vlct.hip), also used by the adjoint to
// recompute the forward intermediates
int launch_prims(const Geom &g, const StateP &st, const Prims &P, uint32_t *status,
                 hipStream_t s);
int launch_fluxes(const Geom &g, const StateP &st, const Prims &P, const Flux &F, int recon,
                  uint32_t *status, hipStream_t s);
int launch_ct(const Geom &g, bool full, const Prims &P, const Flux &F, const StateP &base,
              const StateW &out, const double *dt_dev, uint32_t *status, hipStream_t s);
// upwind sides of the interior faces of F, per axis
int launch_pack_sides(const Geom &g, const Flux &F, uint8_t *const side[3], hipStream_t s);

}  // namespace vlct
