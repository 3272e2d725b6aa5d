/*
 * vlct.h -- C ABI of the MI355X (gfx950) library that advances 3D ideal MHD by
 * one Van Leer + Constrained Transport (VL+CT) time step, following Caddy &
 * Schneider, "Cholla-MHD", Sec. 2.2 (Steps 1-10):
 *
 *   predictor : PCM interface states + HLLD fluxes (Steps 2-3), CT edge
 *               electric fields (Step 4), half-step update to t + dt/2 (Step 5);
 *   corrector : PLMC or PPMC characteristic reconstruction of the half-step
 *               state (Step 6), HLLD fluxes (Step 7), CT edge fields with the
 *               half-step reference field (Step 8), full update from t to
 *               t + dt (Step 9);
 *   next dt   : CFL condition of the updated state (Step 1, Eq. dt), reduced
 *               over the grid on the device.
 *
 * The problem statement follows the paper: conserved cell-centred variables
 * plus face-centred magnetic field, gamma, cell widths and dt go in; the
 * updated state and the next dt come out.
 *
 * Memory: every pointer in vlct_state, dt/next_dt/status and the workspace are
 * DEVICE pointers owned by the caller; the library allocates nothing and never
 * synchronises with the host inside vlct_step / vlct_cfl_dt.  All work is
 * enqueued on `stream` (a hipStream_t; NULL = the default stream) and is
 * stream-ordered, so a call can be captured into a HIP graph.  Arrays are
 * FP64, C order [k][j][i] with x fastest:
 *
 *   rho, mx, my, mz, E : nz*ny*nx        cell averages (density, momentum, total energy)
 *   bx                 : nz*ny*(nx+1)    B_x on x-face i-1/2 of cell i, i = 0..nx
 *   by                 : nz*(ny+1)*nx    B_y on y-face j-1/2, j = 0..ny
 *   bz                 : (nz+1)*ny*nx    B_z on z-face k-1/2, k = 0..nz
 *
 * Each face stores only its normal field component (staggered mesh, Sec. 2.2).
 * Units have mu0 = 1; E = P/(gamma-1) + rho v^2/2 + B^2/2 with the cell-centred
 * field taken as the average of the two face values (Sec. 2.1, Step 1).
 *
 * Boundaries (per axis): periodic, or outflow (zero gradient: cell and
 * transverse-face indices clamp into the grid, normal-face indices clamp into
 * [0, n]).  On a periodic axis the last face plane duplicates the first: its
 * input value is ignored and its output is written equal to face 0.
 *
 * Errors: functions return VLCT_OK or a VLCT_E* code and never abort.  Problems
 * that arise inside kernels (a floor applied, a non-finite result) are OR-ed
 * into *status_dev as VLCT_STATUS_* bits when status_dev is not NULL.
 */
#ifndef VLCT_H
#define VLCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define VLCT_OK 0
#define VLCT_EINVAL 1        /* bad grid descriptor, NULL pointer, unknown option */
#define VLCT_EWORKSPACE 2    /* workspace NULL or smaller than vlct_workspace_bytes() */
#define VLCT_EHIP 3          /* a HIP launch or runtime call failed */
#define VLCT_EUNSUPPORTED 4  /* valid request this build does not implement */
#define VLCT_ESCRATCH 5      /* vlct_step_noalloc: the grid's workspace exceeds the static scratch */

/* corrector reconstruction (Sec. 2.2 Step 6) */
#define VLCT_RECON_PCM 1     /* first order (debugging mode of Step 2) */
#define VLCT_RECON_PLMC 2    /* piecewise linear, limited in characteristic variables */
#define VLCT_RECON_PPMC 3    /* piecewise parabolic, limited in characteristic variables */
#define VLCT_RECON_PLMP 4    /* piecewise linear, limited in primitive variables */
#define VLCT_RECON_PPMP 5    /* piecewise parabolic, limited in primitive variables */

/* boundary condition per axis */
#define VLCT_BC_PERIODIC 0
#define VLCT_BC_OUTFLOW 1

/* bits OR-ed into *status_dev */
#define VLCT_STATUS_PRESSURE_FLOOR 1u  /* a derived or reconstructed pressure was floored */
#define VLCT_STATUS_DENSITY_FLOOR 2u   /* a derived or reconstructed density was floored */
#define VLCT_STATUS_NONFINITE 4u       /* the updated state holds a NaN or Inf */

typedef struct vlct_grid {
    int32_t nx, ny, nz;  /* interior cells per axis, 1 <= n <= 4096 */
    double dx, dy, dz;   /* cell widths, > 0 */
    double gamma;        /* adiabatic index, > 1 */
    double cfl;          /* Courant number, 0 < cfl <= 0.5 (Sec. 2.2 Step 1) */
    int32_t recon;       /* VLCT_RECON_* */
    int32_t bc[3];       /* VLCT_BC_* for x, y, z */
} vlct_grid;

typedef struct vlct_state {
    double *rho, *mx, *my, *mz, *E; /* device, nz*ny*nx each */
    double *bx, *by, *bz;           /* device, face layouts above */
} vlct_state;

/* Bytes of device workspace vlct_step / vlct_cfl_dt need for this grid
 * (0 if the descriptor is invalid).  The workspace holds the half-step state,
 * ghost-padded primitives and face fluxes; its contents are scratch between
 * calls. */
size_t vlct_workspace_bytes(const vlct_grid *g);

/* CFL time step of state `s` (Sec. 2.2 Step 1, Eq. dt):
 *   dt = cfl / max_cells max_l (|v_l| + c_f,l) / d_l,
 * c_f,l the fast magnetosonic speed from cell-centred values with B_l as the
 * longitudinal field.  Writes one double to dt_dev.  Deterministic. */
int vlct_cfl_dt(const vlct_grid *g, const vlct_state *s, double *dt_dev, void *ws,
                size_t ws_bytes, void *stream);

/* One VL+CT step of size *dt_dev from `in` to `out` (Sec. 2.2 Steps 2-9).
 * `out` may alias `in` (all eight pointers equal) or be disjoint from it;
 * any other overlap of an output array with an input array, or of two
 * output arrays, as address ranges of the field sizes above, is VLCT_EINVAL.  next_dt_dev (nullable) receives the CFL
 * step of the result; status_dev (nullable) accumulates VLCT_STATUS_* bits and
 * is never cleared by the library.  dt is read on the device, so a chain of
 * steps needs no host round trip: pass the previous call's next_dt_dev as the
 * next call's dt_dev. */
int vlct_step(const vlct_grid *g, const vlct_state *in, const vlct_state *out,
              const double *dt_dev, double *next_dt_dev, uint32_t *status_dev, void *ws,
              size_t ws_bytes, void *stream);

/* --- stepping without any allocation ---------------------------------------
 * For callers that cannot allocate device memory at all, not even once up
 * front (code under HIP graph capture that owns no buffers, tight serving
 * loops, harnesses that forbid hipMalloc): vlct_step with the workspace taken
 * from a static device array of VLCT_NOALLOC_SCRATCH_BYTES bytes inside the
 * library (one per GPU, held from the library's load until the process ends).
 * Same kernels, same results bit for bit as vlct_step with a caller workspace.
 * The caller still passes the state, dt, next dt and status (device pointers,
 * rules as for vlct_step).  Grids whose vlct_workspace_bytes() exceeds
 * VLCT_NOALLOC_SCRATCH_BYTES (about 55^3 cells on a periodic cube) get
 * VLCT_ESCRATCH before anything is launched.  The scratch of the CURRENT
 * device (hipGetDevice) is used, so `stream` must belong to that device; its
 * address is looked up once per device on the first call there.  Calls
 * share that device's scratch: two calls that overlap in time on one GPU
 * (different streams, or different host threads without ordering) race and
 * give wrong results; calls ordered on one stream are safe.  Allocates
 * nothing (no hipMalloc, hipFree or allocating library routine). */
#define VLCT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int vlct_step_noalloc(const vlct_grid *g, const vlct_state *in, const vlct_state *out,
                      const double *dt_dev, double *next_dt_dev, uint32_t *status_dev,
                      void *stream);

/* --- batched ensembles ----------------------------------------------------
 * Independent instances (own sizes, gamma, cfl, boundaries, dt and state)
 * advanced by one step together: each kernel of the step is launched once for
 * all instances, which fills the GPU when the grids are small.  Every instance
 * computes exactly what vlct_step computes for it (bit-identical results).
 *
 * Bytes of device workspace vlct_step_batch needs for these `count` grid
 * descriptors (host array), 0 if count < 1, count > 65536 or a descriptor is
 * invalid.  The workspace holds a table of the instances and each instance's
 * own workspace; its contents are scratch between calls. */
size_t vlct_batch_workspace_bytes(const vlct_grid *grids, int count);

/* One VL+CT step of every instance i in [0, count): grids[i], in[i], out[i]
 * are HOST arrays of descriptors (the vlct_state members are device
 * pointers); dt_dev, next_dt_dev (nullable) and status_dev (nullable) are
 * DEVICE arrays of `count` elements, instance i using element i.  All
 * instances must use the same reconstruction (else VLCT_EUNSUPPORTED).  Each
 * instance is either fully in place (out[i] == in[i] field by field) or uses
 * output arrays no other array of the call uses (else VLCT_EINVAL).  Returns
 * VLCT_EWORKSPACE if ws_bytes < vlct_batch_workspace_bytes(grids, count).
 * Stream-ordered; no allocation and no host synchronisation. */
int vlct_step_batch(int count, const vlct_grid *grids, const vlct_state *in,
                    const vlct_state *out, const double *dt_dev, double *next_dt_dev,
                    uint32_t *status_dev, void *ws, size_t ws_bytes, void *stream);

/* Per-instance tile plan: vlct_step_batch with plan[i] (HOST array of `count`
 * bytes, NULL = all zero) choosing instance i's tiles: low nibble the CT
 * column tile (0: 64 x 8, 1: 32 x 16, 2: 16 x 32), high nibble the corrector
 * march segment along y and z (0: 16 faces, 1: 32, 2: 8).  Plan 0 takes
 * 64 x 8 CT tiles with vlct_step's planes per CT block and 16-face marches
 * (vlct_step itself marches 8 faces on small grids).  Every plan gives the
 * same results bit for bit (the tiles only regroup the same per-cell and
 * per-face arithmetic); VLCT_EINVAL for an unknown variant. */
int vlct_step_batch_plan(int count, const vlct_grid *grids, const vlct_state *in,
                         const vlct_state *out, const double *dt_dev, double *next_dt_dev,
                         uint32_t *status_dev, const uint8_t *plan, void *ws, size_t ws_bytes,
                         void *stream);

/* Ensembles with per-instance end times (each run to its own t_end): one step
 * of vlct_step_batch_plan for every instance still running, in place
 * (states[i] is both input and output).  Instance i is running while
 * t_dev[i] < t_end_dev[i]; it then advances by min(dt_dev[i],
 * t_end_dev[i] - t_dev[i]) (its last step clipped to land on t_end), writes
 * its next CFL step to next_dt_dev[i] and adds the step to t_dev[i].  A
 * finished instance's blocks return at once in every kernel, so it costs
 * almost nothing while the others continue, and its state, time and dt stay
 * as they are.  t_dev (device, read and written), t_end_dev (device, read),
 * next_dt_dev (device, required: VLCT_EINVAL if NULL); the other arguments
 * as for vlct_step_batch_plan.  Everything happens on the device, so a loop of
 * these calls needs no host synchronisation (check t_dev now and then).  An
 * instance's result is bitwise that of vlct_step applied with the same clip
 * (dt = min(dt, t_end - t), t += dt). */
int vlct_step_batch_until(int count, const vlct_grid *grids, const vlct_state *states,
                          const double *dt_dev, double *next_dt_dev, uint32_t *status_dev,
                          double *t_dev, const double *t_end_dev, const uint8_t *plan, void *ws,
                          size_t ws_bytes, void *stream);

/* Autotuner for a batch: writes into plan[count] (host) the tiles that make
 * the batched step fastest, found by timing it on this batch: instances are
 * grouped by nx (<= 24, <= 48, <= 96, larger) and each group's CT tile, then
 * its march segment, is changed while the rest of the batch keeps its current
 * choice, keeping a change that makes the whole step at least 1% faster.
 * Each trial times `reps` (1..100) batched steps after one untimed step.  The
 * trial steps read `in` and overwrite `out` (every instance must be out of
 * place, else VLCT_EINVAL; next dt and status are not written).  Unlike the
 * step calls, this call synchronises with the host (it creates and destroys
 * two HIP events) and must not be captured into a graph. */
int vlct_batch_tune(int count, const vlct_grid *grids, const vlct_state *in,
                    const vlct_state *out, const double *dt_dev, void *ws, size_t ws_bytes,
                    void *stream, int reps, uint8_t *plan);

/* --- adjoint of one step --------------------------------------------------
 * Reverse derivative of the VL+CT step of Sec. 2.2 (Steps 2-9) at the state
 * `in`, for the step size *dt_dev held fixed:
 *     lam_in = (d out / d in)^T lam_out
 * where `out` is what vlct_step(g, in, out, dt_dev, ...) writes.  Each state
 * element (cells and every stored face, the periodic duplicate face
 * included) is one coordinate: lam_out and lam_in use the vlct_state layout
 * of the state.  The output's duplicate face n is a copy of face 0, so its
 * cotangent acts on face 0; the step never reads the input's duplicate face,
 * so lam_in is zero there.  Every branch of the step (HLLD wave regions,
 * limiter cases, CT upwind sides, floors) is taken as in the forward step at
 * `in`; at a branch boundary the result is the one-sided derivative of the
 * branch taken.
 *
 * Bytes of device workspace vlct_step_adjoint needs for this grid (0 if the
 * descriptor is invalid).  The workspace holds the forward intermediates
 * (primitives, fluxes, half-step state) and the cotangents of each stage. */
size_t vlct_adjoint_workspace_bytes(const vlct_grid *g);

/* Writes lam_in (device arrays, none shared with `in` or `lam_out`, else
 * VLCT_EINVAL).  in, lam_out: device, read only.  dt_dev: device pointer to
 * the step size.  Periodic boundaries on every axis only (else
 * VLCT_EUNSUPPORTED); every corrector reconstruction.  VLCT_EWORKSPACE if
 * ws_bytes < vlct_adjoint_workspace_bytes(g).  Stream-ordered; no
 * allocation and no host synchronisation.  Not bit-reproducible from run to
 * run: where a cell gathers cotangents from the reconstructions of several
 * faces they are summed with FP64 atomics, whose order of addition varies,
 * so two runs on the same input differ at rounding level. */
int vlct_step_adjoint(const vlct_grid *g, const vlct_state *in, const vlct_state *lam_out,
                      const vlct_state *lam_in, const double *dt_dev, void *ws, size_t ws_bytes,
                      void *stream);

/* --- taped steps ----------------------------------------------------------
 * A taped step is vlct_step (same kernels, same results bit for bit) that
 * also keeps, in a caller-owned device buffer, what the adjoint would
 * otherwise recompute: the half-step state U^{n+1/2} and the upwind side of
 * every face of both stages (one byte each).  The adjoint of that step can
 * then skip the recomputation of the fluxes.
 *
 * Bytes of one step's tape (0 if the descriptor is invalid). */
size_t vlct_tape_bytes(const vlct_grid *g);

/* vlct_step (same arguments and rules) writing the step's tape to `tape`
 * (device, tape_bytes >= vlct_tape_bytes(g), else VLCT_EWORKSPACE).  The tape
 * stays valid while `in` is unchanged. */
int vlct_step_taped(const vlct_grid *g, const vlct_state *in, const vlct_state *out,
                    const double *dt_dev, double *next_dt_dev, uint32_t *status_dev, void *ws,
                    size_t ws_bytes, void *tape, size_t tape_bytes, void *stream);

/* Bytes of device workspace vlct_step_adjoint_taped needs (0 if invalid). */
size_t vlct_adjoint_taped_workspace_bytes(const vlct_grid *g);

/* vlct_step_adjoint for the step vlct_step_taped(g, in, ..., dt_dev, ...)
 * wrote `tape` for (same in, same *dt_dev): same result (up to the summation
 * order of accumulations), without recomputing the step's fluxes.  tape:
 * device, read only.  Same argument rules and codes as vlct_step_adjoint;
 * VLCT_EWORKSPACE also for a short tape. */
int vlct_step_adjoint_taped(const vlct_grid *g, const vlct_state *in, const vlct_state *lam_out,
                            const vlct_state *lam_in, const double *dt_dev, const void *tape,
                            size_t tape_bytes, void *ws, size_t ws_bytes, void *stream);

/* Face fields of an edge-centred vector potential, B = curl_h A, on a periodic
 * grid (the vertex/edge potential of the CT scheme, Sec. 2.2; its discrete
 * divergence vanishes to rounding).  ax[k][j][i] sits at (i, j-1/2, k-1/2),
 * ay at (i-1/2, j, k-1/2), az at (i-1/2, j-1/2, k); each is a device array of
 * nz*ny*nx doubles.  bx, by, bz: device face arrays in the vlct_state layout,
 * written completely (the duplicate periodic plane n equals plane 0).
 * VLCT_EUNSUPPORTED unless every axis is periodic. */
int vlct_curl_potential(const vlct_grid *g, const double *ax, const double *ay, const double *az,
                        double *bx, double *by, double *bz, void *stream);

/* Transpose of vlct_curl_potential: (lax, lay, laz) = curl_h^T (lbx, lby, lbz),
 * with the cotangent of each duplicate face plane acting on plane 0 (the face
 * it copies).  Overwrites lax, lay, laz; device arrays; periodic only. */
int vlct_curl_potential_adjoint(const vlct_grid *g, const double *lbx, const double *lby,
                                const double *lbz, double *lax, double *lay, double *laz,
                                void *stream);

/* --- diagnostics ----------------------------------------------------------
 * vlct_step_observed is vlct_step (same arguments, rules, kernels and results)
 * that invokes cb(user, kernel, phase, stream) on the calling host thread
 * immediately before (phase 0) and after (phase 1) it enqueues each kernel,
 * with the stream the kernel goes to, so a profiler can bracket one kernel
 * family with events on that stream.  `kernel` is a VLCT_KERNEL_* id.  The
 * observer belongs to this call alone: no state outlives it or is visible to
 * other threads.  cb must not be NULL (VLCT_EINVAL). */
#define VLCT_KERNEL_PRIMS 0        /* primitive variables (both stages) */
#define VLCT_KERNEL_FLUX_PCM 1     /* predictor: PCM states + HLLD, one launch per axis */
#define VLCT_KERNEL_FLUX_RECON 2   /* corrector: PLMC/PPMC states + HLLD, one launch per axis */
#define VLCT_KERNEL_EDGES 3        /* reserved (edge fields are computed inside the updates) */
#define VLCT_KERNEL_UPDATE_HALF 4  /* CT edge fields + half-step cell and face update */
#define VLCT_KERNEL_UPDATE_FULL 5  /* CT edge fields + full-step cell and face update */
#define VLCT_KERNEL_DT 6           /* CFL reduction over a state (two launches: vlct_cfl_dt, in-place steps) */
#define VLCT_KERNEL_DT_FINAL 7     /* last launch of a step's CFL reduction whose per-block
                                      maxima the full update computed */
#define VLCT_KERNEL_PREDICTOR 8    /* the whole predictor of a step: primitives, PCM HLLD
                                      fluxes, CT edge fields and half-step update in one kernel */
#define VLCT_KERNEL_COUNT 9
typedef void (*vlct_launch_observer)(void *user, int kernel, int phase, void *stream);
int vlct_step_observed(const vlct_grid *g, const vlct_state *in, const vlct_state *out,
                       const double *dt_dev, double *next_dt_dev, uint32_t *status_dev, void *ws,
                       size_t ws_bytes, void *stream, vlct_launch_observer cb, void *user);

/* Name of a VLCT_KERNEL_* id ("?" if unknown). */
const char *vlct_kernel_name(int kernel);

/* Static description of a return code. */
const char *vlct_strerror(int code);

/* ABI version of this header (major*100 + minor). */
int vlct_abi_version(void);

#define VLCT_ABI_VERSION 100

#ifdef __cplusplus
}
#endif
#endif /* VLCT_H */
