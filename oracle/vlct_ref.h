/*
 * vlct_ref.h -- interface of the CPU oracle for one Van Leer + Constrained
 * Transport (VL+CT) step of 3D ideal MHD (Caddy & Schneider, "Cholla-MHD",
 * Sec. 2.1-2.2).
 *
 * TEST INFRASTRUCTURE ONLY. This oracle exists to check the GPU library; it
 * shares no code, header or table with it. Only the test-suite, the smoke
 * entry point and the benchmark's CPU-baseline leg may load it.
 *
 * All pointers are host pointers. Arrays are C order [k][j][i] (x fastest):
 *   rho, mx, my, mz, E : nz*ny*nx          cell averages
 *   bx                 : nz*ny*(nx+1)      x-face i-1/2 of cell i, i = 0..nx
 *   by                 : nz*(ny+1)*nx      y-face j-1/2, j = 0..ny
 *   bz                 : (nz+1)*ny*nx      z-face k-1/2, k = 0..nz
 * On a periodic axis the last face plane duplicates the first: its input
 * value is ignored and its output is a copy of face 0.
 */
#ifndef VLCT_REF_H
#define VLCT_REF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;   /* interior cells per axis, >= 1 */
    double dx, dy, dz;    /* cell widths, > 0 */
    double gamma;         /* adiabatic index, > 1 */
    double cfl;           /* Courant number in (0, 0.5] */
    int32_t recon;        /* corrector reconstruction: 1 PCM, 2 PLMC, 3 PPMC, 4 PLMP, 5 PPMP */
    int32_t bc[3];        /* per axis: 0 = periodic, 1 = outflow (zero gradient) */
} vref_grid;

/* Status bits OR-ed into *status by the step. */
#define VREF_STATUS_PRESSURE_FLOOR 1u
#define VREF_STATUS_DENSITY_FLOOR 2u
#define VREF_STATUS_NONFINITE 4u

/* Return codes. */
#define VREF_OK 0
#define VREF_EINVAL 1

/* One full VL+CT step of size dt. in[8] = {rho,mx,my,mz,E,bx,by,bz};
 * out may alias in. next_dt (nullable) receives the CFL step of the result. */
int vref_step(const vref_grid *g, const double *const in[8], double *const out[8],
              double dt, double *next_dt, uint32_t *status, int nthreads);

/* CFL time step of a state (Sec. 2.2 Step 1, Eq. dt). */
int vref_cfl_dt(const vref_grid *g, const double *const st[8], double *dt, int nthreads);

/* --- unit-level entry points used by the oracle's own pins ----------------- */

/* Fast and slow magnetosonic speeds of a primitive state with normal field bn. */
void vref_wave_speeds(double rho, double p, double bn, double bt1, double bt2,
                      double gamma, double *cf, double *cs);

/* HLLD flux.  w = (rho, v_n, v_t1, v_t2, P, B_t1, B_t2) in the sweep frame,
 * bn the face-normal field.  flux[0..6] = (rho, m_n, m_t1, m_t2, E, B_t1, B_t2);
 * flux[7] = upwind indicator (+1, -1 or 0) used by the CT edge EMFs. */
void vref_hlld(const double wl[7], const double wr[7], double bn, double gamma,
               double flux[8]);

/* Physical flux of a primitive state in the sweep frame (Sec. 2.1). */
void vref_phys_flux(const double w[7], double bn, double gamma, double flux[7]);

/* Eigen-system of the 1D primitive system at state w with normal field bn.
 * R: right eigenvectors as columns (row-major 7x7), L = R^{-1},
 * lam: eigenvalues in order u-cf, u-ca, u-cs, u, u+cs, u+ca, u+cf. */
void vref_eigen(const double w[7], double bn, double gamma, double R[49], double L[49],
                double lam[7]);

/* Reconstruction of one cell along one sweep: stencil w[(2r+1)*7] centred on
 * the cell (r = 1 for PLMC, 2 for PPMC), bn = cell-centred normal field.
 * face_minus = state at the cell's low face (right state of face i-1/2),
 * face_plus  = state at the cell's high face (left state of face i+1/2). */
void vref_plmc(const double w[21], double bn, double gamma, double face_minus[7],
               double face_plus[7]);
void vref_ppmc(const double w[35], double bn, double gamma, double face_minus[7],
               double face_plus[7]);
/* primitive-variable limiting: the same steps without the characteristic projections */
void vref_plmp(const double w[21], double face_minus[7], double face_plus[7]);
void vref_ppmp(const double w[35], double bn, double gamma, double face_minus[7],
               double face_plus[7]);

/* Conservative face update of B from edge EMFs (Sec. 2.2 Step 5/9 CT update):
 * ex: (nz+1)*(ny+1)*nx at (i, j-1/2, k-1/2); ey: (nz+1)*ny*(nx+1) at
 * (i-1/2, j, k-1/2); ez: nz*(ny+1)*(nx+1) at (i-1/2, j-1/2, k).
 * b_out = b_in - dt * curl(E) on every stored face. */
void vref_ct_update(const vref_grid *g, const double *const b_in[3], double *const b_out[3],
                    const double *ex, const double *ey, const double *ez, double dt);

/* Edge EMFs of one stage from a state (diagnostic / pins): computes the stage
 * fluxes with the given reconstruction (1 = PCM, 2 = PLMC, 3 = PPMC) and
 * returns the CT edge EMFs in the vref_ct_update layout. */
int vref_edge_emfs(const vref_grid *g, const double *const st[8], int recon, double *ex,
                   double *ey, double *ez, int nthreads);

/* Predictor only (Steps 2-5): writes the half-step state of a step of size dt
 * to out (must not alias in). */
int vref_half_step(const vref_grid *g, const double *const in[8], double *const out[8],
                   double dt, int nthreads);

/* Face fluxes of one stage (diagnostics): 7 sweep-frame components + upwind
 * indicator per face of each axis, in the face layout of that axis. */
int vref_stage_fluxes(const vref_grid *g, const double *const st[8], int recon,
                      double *const Fx[8], double *const Fy[8], double *const Fz[8],
                      int nthreads);

/* max over cells of |div B| * dx / max|B_cc|  (normalised divergence). */
double vref_divb_norm(const vref_grid *g, const double *const st[8]);

#ifdef __cplusplus
}
#endif
#endif
