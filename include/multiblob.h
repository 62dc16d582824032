/*
 * multiblob.h -- C ABI of the MI355X (gfx950) multiblob immersed-boundary
 * step.
 *
 * Method: Vazquez-Quesada, Balboa Usabiaga, Delgado-Buscalioni, "A multiblob
 * approach to colloidal hydrodynamics with inherent lubrication",
 * arXiv:1407.5600.  A particle is a set of blobs (12 on the vertices of an
 * icosahedron plus one at its centre) held together by harmonic springs
 * (Fig. 1).  Blob i couples to the fluid through the kernel delta_h of
 * eq. delta: interpolation u_i = J_i v (eq. ju), spreading S_i = J_i^*, and
 * the fluid obeys eq. vf with the solenoidal projector P.
 *
 * Discretisation used by every call:
 *   - periodic cube of L^3 cells of side h;
 *   - staggered (MAC) velocity: component a of node (i,j,k) lives at
 *     h*(i,j,k) + (h/2) e_a;
 *   - delta_h(r) = h^-3 prod_a Phi(r_a / h) with the 3-point function Phi
 *     fixed by the moment conditions stated after eq. delta;
 *   - fluid solve: Crank-Nicolson for the viscous term, or steady Stokes,
 *     with exact projection, solved by FFT on the MAC grid (the convective
 *     and fluctuating stresses of eq. vf are not included).
 *
 * Memory: every pointer argument except those marked "host" is a device
 * pointer on the grid's device, aligned to 256 bytes (as every hipMalloc
 * and torch allocation is); a misaligned pointer gives MB_ERR_INVALID.  The
 * caller owns all buffers; the library never frees them and keeps none
 * beyond the call, except a workspace given to mb_grid_set_workspace.
 * Layouts:
 *   q, F, u     [M][3] float64, row-major; blob nb*p + b belongs to
 *               particle p (b = 0..11 vertices, 12 the centre).
 *   Fext, U0    [P][3] float64.
 *   fields      [3][L][L][L], x fastest; float64 for MB_FP64 grids,
 *               float32 for MB_MIXED grids.  f is a force density.
 *   Positions are unwrapped (any real value); only indices are wrapped.
 *
 * Streams: `stream` is a hipStream_t (NULL = default stream).  Every call
 * only enqueues work on that stream and returns; errors found while
 * enqueueing are returned, device faults surface at a later
 * synchronisation.  One grid must not be used from two streams or threads
 * at once (it owns scratch buffers).
 *
 * Errors: every call returns an mb_status and never throws.  Invalid
 * arguments (null or misaligned pointers, sizes out of range, a grid from
 * another device, a grid without its workspace) give MB_ERR_INVALID; a
 * valid configuration this library has no kernels for gives
 * MB_ERR_UNSUPPORTED; no usable GPU, a failed launch or a device error
 * reported while enqueueing gives MB_ERR_DEVICE; allocation failure gives
 * MB_ERR_NOMEM; with check_finite, a non-finite blob position or force
 * gives MB_ERR_NONFINITE (see mb_grid_desc).
 */
#ifndef MULTIBLOB_H
#define MULTIBLOB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MB_OK = 0,
    MB_ERR_INVALID = -1,
    MB_ERR_UNSUPPORTED = -2,
    MB_ERR_NOMEM = -3,
    MB_ERR_DEVICE = -4,
    MB_ERR_NONFINITE = -5
} mb_status;

typedef enum {
    MB_FP64 = 0,  /* every field and accumulation in float64 */
    MB_MIXED = 1  /* fields, kernel weights, FFT and accumulation in float32;
                     positions, spring forces, the k = 0 mode and momentum
                     reductions in float64 */
} mb_precision;

typedef enum {
    MB_UNSTEADY_CN = 0,   /* rho dv/dt = eta L v - grad pi + f (eq. vf at
                             zero Reynolds number), Crank-Nicolson */
    MB_STEADY_STOKES = 1  /* 0 = eta L v - grad pi + f, mean(v) = 0 (the
                             Stokes limit used for the paper's viscosity
                             runs, Sec. Stresslet and viscosity) */
} mb_mode;

typedef enum {
    MB_SCHEME_EULER = 0,    /* first order (the default): the forces, the
                               spreading and the interpolation at q^n, the
                               blobs moved by dt J(q^n) v^{n+1} */
    MB_SCHEME_MIDPOINT = 1  /* second order: a midpoint predictor-corrector
                               rebuilt from eqs. vf, ju and blob1 with m_e =
                               0 (the inertial coupling scheme the paper
                               uses is cited, not printed):
                               q* = q^n + (dt/2) J(q^n) v^n;  v^{n+1} from
                               v^n with f = S(q*) F(q*);  q^{n+1} = q^n +
                               dt J(q*) (v^n + v^{n+1})/2.  In
                               MB_STEADY_STOKES the explicit midpoint rule
                               with a steady solve at q^n and one at q*. */
} mb_scheme;

/* Grid description.
 *
 * L: cells per side, 8 <= L <= 512, L = 2^a 3^b (the FFT plans are radix 2,
 * 3, 4, 8 and 16, compiled per size), and L a multiple of 8: the binning,
 * spreading and interpolation kernels work on tiles of 8 or 16 cells per
 * axis (tile indices by shifts, one workgroup per tile).  The sizes with
 * kernels are 8, 16, 24, 32, 48, 64, 72, 96, 128, 144, 192, 216, 256, 288,
 * 384, 432 and 512; other 2^a 3^b sizes (12, 18, 27, 36, 54, 81, 108, ...)
 * give MB_ERR_UNSUPPORTED, any other L MB_ERR_INVALID.
 * h > 0, dt > 0; rho > 0 in MB_UNSTEADY_CN; eta > 0 in MB_STEADY_STOKES
 * (eta = 0 is allowed in MB_UNSTEADY_CN: ideal fluid).  zero_mean = 1 holds
 * the k = 0 velocity mode at zero (a periodic array of particles with no net
 * flow, the setting of eq. rhinf); zero_mean = 0 evolves it exactly,
 * mean(v') = mean(v) + (dt/rho) mean(f).  max_blobs bounds the M of every
 * later call on this grid (blob-sized scratch is sized once).
 *
 * deterministic = 1: every result is the same bit for bit from run to run.
 * Spreading always sums in fixed point (independent of the order of the
 * blobs and of the atomic additions); the one order-dependent path, float64
 * LDS atomics for a float64 spreading box tile (16^3 cells) of more than
 * 2^20 blobs, is then replaced by two 64-bit fixed-point sums (the
 * contributions, then their rounding remainders; up to 2^25 blobs in one
 * box tile, beyond which the atomics remain), and mb_step_adjoint sums the
 * stiffness and rest-length derivatives per block in a fixed order instead
 * of with float64 atomics.  deterministic = 0 allows those paths.
 *
 * check_finite = 1: the calls that read blob positions or blob forces
 * (mb_spread, mb_interpolate, mb_interpolate_grad and every step call)
 * check each position and force they use, at every step; if one is NaN or
 * infinite the call finishes its launches, waits for its stream and
 * returns MB_ERR_NONFINITE (its outputs are then undefined).  The check
 * costs one stream synchronisation per call, so mb_step_graph checks only
 * after its last replay.  check_finite = 0 (the default): no check and no
 * synchronisation; non-finite inputs give non-finite or meaningless
 * outputs, never an access outside the library's buffers.
 * The same check reports a stalled scan: in a step the first workgroup of
 * the spring-force kernel sums the tile counts and the others wait for it,
 * for at most one to two seconds (only a device that does not run that
 * workgroup makes them give up); a workgroup that gives up writes no
 * records, and with check_finite = 1 the call returns MB_ERR_DEVICE, with
 * check_finite = 0 its outputs are undefined.
 *
 * external_workspace = 1: mb_grid_create allocates no scratch; every call
 * on the grid returns MB_ERR_INVALID until a workspace of at least
 * mb_workspace_size bytes is given with mb_grid_set_workspace (for example
 * a torch tensor, so that one allocator holds all device memory). */
typedef struct {
    int32_t L;
    int32_t precision; /* mb_precision */
    int32_t mode;      /* mb_mode */
    int32_t zero_mean;
    double h;
    double rho;
    double eta;
    double dt;
    int64_t max_blobs;
    int32_t deterministic;
    int32_t check_finite;
    int32_t external_workspace;
    int32_t reserved;  /* must be 0 */
} mb_grid_desc;

typedef struct mb_grid mb_grid;       /* opaque; owns FFT tables and scratch */
typedef struct mb_springs mb_springs; /* opaque; owns the pair table */

/* Create a grid on the current HIP device.  Unless desc->external_workspace
 * is set, allocates its workspace (mb_workspace_size bytes: the FFT tables,
 * the spectrum of about 1.5 L^3 complex values, the spread boxes of about
 * 5-7 L^3 values of the field precision, the per-tile binning arrays and
 * ~100 B per blob), which it frees at mb_grid_destroy.  *out is set to NULL
 * on error. */
mb_status mb_grid_create(const mb_grid_desc* desc, mb_grid** out);

/* Bytes of device workspace a grid of this description holds (nbox boxes;
 * nbox = 1 for mb_grid_create): the FFT twiddle and symbol tables, the
 * spectrum, the spread boxes (sized for every tile shape that fits L, so
 * mb_grid_set_tiles and mb_grid_autotune never reallocate), the binning
 * arrays, the sorted blob records and the partial sums of the diagnostics.
 * The midpoint scheme (mb_grid_set_scheme), forced steps and the reverse
 * step keep their extra scratch outside it (allocated by the library when
 * first enabled or called).  0 for an invalid description or nbox. */
size_t mb_workspace_size(const mb_grid_desc* desc, int32_t nbox);

/* Give the grid a caller-owned device workspace of `bytes` bytes (at least
 * mb_workspace_size of the grid's description and box count, 256-byte
 * aligned, on the grid's device), replacing the workspace it had (a
 * library-allocated one is freed).  Waits for the device first (no work of
 * this grid may be in flight), then initialises the workspace (FFT tables,
 * zeroed counters) on the NULL stream and waits for that.  The caller must
 * keep the buffer alive and unused by anything else until mb_grid_destroy
 * or the next mb_grid_set_workspace.  The sorted order of the last binning
 * is forgotten (results are unchanged).  MB_ERR_INVALID if dev_ptr is NULL
 * or misaligned, or bytes too small. */
mb_status mb_grid_set_workspace(mb_grid* grid, void* dev_ptr, size_t bytes);

/* A grid holding a batch of nbox independent periodic boxes of the same
 * description (1 <= nbox <= 65536), each call advancing all of them in one
 * launch per kernel: the pair-mobility sweeps of the paper's lubrication and
 * pass-by set-ups run many small boxes at once.  Layouts in every call on
 * such a grid: fields [nbox][3][L][L][L]; blob arrays [nbox * Mb][3] with
 * box b holding blobs b*Mb .. b*Mb+Mb-1 (the same Mb in every box; calls
 * reject M not divisible by nbox); particle arrays likewise (P divisible by
 * nbox).  max_blobs counts the blobs of all boxes.  Diagnostics of mb_step
 * sum over the boxes.  mb_grid_create is the case nbox = 1. */
mb_status mb_grid_create_batch(const mb_grid_desc* desc, int32_t nbox,
                               mb_grid** out);

/* Release a grid and the workspace it allocated (synchronises its device
 * first; a caller-given workspace is left to the caller).  NULL is
 * accepted. */
mb_status mb_grid_destroy(mb_grid* grid);

/* Spring table of one particle template (Fig. 1: hard springs joining the
 * blobs): npairs pairs (pair_a[e], pair_b[e]) of blob indices in
 * [0, blobs_per_particle) with rest lengths rest_len[e] > 0 and stiffness
 * k >= 0; energy sum_e (k/2)(|q_b - q_a| - rest_len[e])^2 per particle.
 * All three arrays are HOST arrays, copied.  blobs_per_particle <= 64, each
 * blob in at most 63 pairs. */
mb_status mb_springs_create(int32_t blobs_per_particle, int32_t npairs,
                            const int32_t* pair_a, const int32_t* pair_b,
                            const double* rest_len, double k,
                            mb_springs** out);
mb_status mb_springs_destroy(mb_springs* springs);

/* New rest lengths (HOST array of npairs values > 0, read before the call
 * returns and copied to the device in the order of `stream`) and stiffness
 * k >= 0 of a spring table, for every call enqueued after this one (fitting
 * k and the particle size changes them between trajectories without a new
 * table or a device synchronisation). */
mb_status mb_springs_set_params(mb_springs* springs, const double* rest_len,
                                double k, void* stream);

/* Spreading S (definition of S_i after eq. jm): f_out = sum_i
 * delta_h(x - q_i) F_i at every staggered node, overwriting f_out.
 * M blobs (0 <= M <= max_blobs).  q, F: [M][3] float64; f_out: field. */
mb_status mb_spread(mb_grid* grid, int64_t M, const double* q,
                    const double* F, void* f_out, void* stream);

/* Interpolation J (eq. ju): u_out[i] = sum_x h^3 delta_h(x - q_i) v(x).
 * v: field (not modified); u_out: [M][3] float64. */
mb_status mb_interpolate(mb_grid* grid, int64_t M, const double* q,
                         const void* v, double* u_out, void* stream);

/* Fluid solve of eq. vf (mode of the grid) with the solenoidal projection P:
 * v_out = new velocity from v_in and the force density f.  v_in may equal
 * v_out; v_in is unused in MB_STEADY_STOKES (may be NULL there). */
mb_status mb_fluid_solve(mb_grid* grid, const void* v_in, const void* f,
                         void* v_out, void* stream);

/* Spring forces plus the particle's external force split evenly over its
 * blobs: F_out[nb*p + b] = Fext[p]/nb + sum of the springs of blob b.
 * Fext may be NULL (no external force).  q, F_out: [P*nb][3]; Fext [P][3]. */
mb_status mb_spring_forces(const mb_springs* springs, int64_t nparticles,
                           const double* q, const double* Fext,
                           double* F_out, void* stream);

/* nsteps time steps of the coupled system, in place on q and v:
 *   F^n = springs(q^n) + Fext/nb;  f = S(q^n) F^n;  v^{n+1} = solve(v^n, f);
 *   u = J(q^n) v^{n+1};  q^{n+1} = q^n + dt u;
 * (eq. vf with neutrally buoyant blobs, m_e = 0 as in Table 1, so the
 * fluid-blob force is minus the blob force; no-slip u_i = J_i v).
 * u_out [M][3] and U0_out [P][3] (particle velocity U0 = (1/N) sum_i u_i,
 * Sec. Multiblob particle model) receive the last step's values and may be
 * NULL.  diag_out (may be NULL) receives 7 float64 on the device:
 * {Pi_x, Pi_y, Pi_z, sumF_x, sumF_y, sumF_z, max|D v|} of the last step,
 * with Pi = rho h^3 sum_x v after the step (their partial sums are formed
 * on that step only, and only when diag_out is given).  Within one call,
 * each step after the first takes the binning of its blobs from the
 * interpolation of the step before (same results, one kernel fewer); a
 * call always starts by binning q afresh, so q may be changed between
 * calls.  nsteps >= 0. */
mb_status mb_step(mb_grid* grid, const mb_springs* springs,
                  int64_t nparticles, double* q, void* v, const double* Fext,
                  double* u_out, double* U0_out, double* diag_out,
                  int32_t nsteps, void* stream);

/* mb_step with per-blob external forces: F^n = springs(q^n) + Fext/nb +
 * F_blob (F_blob [M][3] float64 on the device, may be NULL; Fext may be
 * NULL).  Used by the differentiable trajectory, whose forcing is per blob. */
mb_status mb_step_ext(mb_grid* grid, const mb_springs* springs,
                      int64_t nparticles, double* q, void* v,
                      const double* Fext, const double* F_blob,
                      double* u_out, double* U0_out, double* diag_out,
                      int32_t nsteps, void* stream);

/* mb_step_ext with a force density f_fluid acting on the fluid besides the
 * spread blob forces: the solve of each step takes f = S(q^n) F^n + f_fluid.
 * It drives the periodic forcing f = f0 sin(k_j y) x of the viscosity
 * measurement (Sec. Stresslet and Viscosity).  f_fluid: [3][L][L][L]
 * ([nbox][3][L][L][L] for a batch), the grid's precision, on the device,
 * not NULL, unchanged by the call.  The first call allocates one field of
 * scratch in the grid (kept until mb_grid_destroy; MB_ERR_NOMEM if that
 * fails).  The diagnostics' sum F covers the blob forces only. */
mb_status mb_step_forced(mb_grid* grid, const mb_springs* springs,
                         int64_t nparticles, double* q, void* v,
                         const double* Fext, const double* F_blob,
                         const void* f_fluid, double* u_out, double* U0_out,
                         double* diag_out, int32_t nsteps, void* stream);

/* mb_spring_forces plus per-blob external forces F_blob [M][3] (may be
 * NULL). */
mb_status mb_spring_forces_ext(const mb_springs* springs, int64_t nparticles,
                               const double* q, const double* Fext,
                               const double* F_blob, double* F_out,
                               void* stream);

/* nsteps steps of each of ngrids grids (as mb_step_ext, no per-step
 * outputs), with one step of every grid captured once into a HIP graph and
 * the graph launched nsteps times on a private stream ordered after
 * `stream`; returns when the steps are done.  Launch-bound workloads (many
 * small boxes, several size classes) then pay one graph launch per step.
 * Arrays per grid as in mb_step_ext (Fext and F_blob entries may be NULL).
 * Grids with no blobs are allowed; timing hooks are off during the capture. */
mb_status mb_step_graph(int32_t ngrids, mb_grid* const* grids,
                        const mb_springs* const* springs,
                        const int64_t* nparticles, double* const* q,
                        void* const* v, const double* const* Fext,
                        const double* const* F_blob, int32_t nsteps,
                        void* stream);

/* ---- Derivatives (reverse mode) of the step, for gradients of losses over
 * trajectories.  They use that J and S are each other's adjoints (Sec.
 * Multiblob particle model: S_i = J_i^*, so J^T = h^3 S), that the fluid
 * solve is self-adjoint (the projection P of eq. vf is Hermitian per
 * wavevector and commutes with the viscous operator), and that the kernel
 * of eq. delta is C^1.  All arrays are float64 device arrays; results are
 * ACCUMULATED into the *_inout / bar arrays (zero them to start). */

/* g_inout[i] += sum_a W[i][a] grad_{q_i} (J_i v)_a: the derivative of the
 * interpolation (eq. ju) with respect to the blob positions contracted with
 * blob weights W [M][3].  v: field in the grid's precision. */
mb_status mb_interpolate_grad(mb_grid* grid, int64_t M, const double* q,
                              const void* v, const double* W, double* g_inout,
                              void* stream);

/* Transposed Jacobian of the spring forces (Fig. 1 springs, energy
 * sum (k/2)(|q_b - q_a| - r0)^2) applied to Fbar [M][3]:
 * qbar += (dF/dq)^T Fbar;  *kbar += Fbar . dF/dk;  r0bar[e] += Fbar .
 * dF/dr0_e summed over particles (kbar: 1 double, r0bar: npairs doubles,
 * each may be NULL).  kbar and r0bar are summed with float64 atomics: their
 * last bits may vary run to run. */
mb_status mb_spring_adjoint(const mb_springs* springs, int64_t nparticles,
                            const double* q, const double* Fbar, double* qbar,
                            double* kbar, double* r0bar, void* stream);

/* Reverse of one mb_step_ext step on a float64 grid (MB_ERR_UNSUPPORTED on
 * a mixed grid).  Inputs: the step's starting positions q_n [M][3], the
 * velocity after its fluid solve v_np1 [3][L^3], its forcing (Fext [P][3],
 * F_blob [M][3], either may be NULL), and ubar_loss [M][3] (may be NULL), the
 * loss gradient with respect to this step's blob velocities u^n.  In/out:
 * qbar [M][3] holds dloss/dq^{n+1} on entry and dloss/dq^n on return; vbar
 * [3][L^3] likewise dloss/dv^{n+1} -> dloss/dv^n.  Accumulated:
 * Fblob_bar [M][3] (dloss/dF_blob), kbar (1 double), r0bar (npairs doubles);
 * each may be NULL.  Allocates its scratch (about 9 L^3 + 9 max_blobs
 * doubles) on the first call. */
mb_status mb_step_adjoint(mb_grid* grid, const mb_springs* springs,
                          int64_t nparticles, const double* q_n,
                          const void* v_np1, const double* Fext,
                          const double* F_blob, const double* ubar_loss,
                          double* qbar, void* vbar, double* Fblob_bar,
                          double* kbar, double* r0bar, void* stream);

/* ---- Allocation-free step, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  mb_step on a first-order grid described by desc (nbox = 1,
 * desc->external_workspace ignored), with the grid's whole workspace in a
 * static device array of MB_NOALLOC_SCRATCH_BYTES held by the library on
 * each GPU it runs on until the process ends: no hipMalloc, hipFree or
 * other allocation.  Inputs, outputs and springs as mb_step (the caller
 * passes them; the springs table is made beforehand with
 * mb_springs_create).  Each call rebuilds the FFT tables and clears the
 * counters in the array on `stream`, by kernels, then steps; results equal
 * mb_step's on a grid of the same description.  MB_ERR_UNSUPPORTED when
 * mb_workspace_size(desc, 1) exceeds MB_NOALLOC_SCRATCH_BYTES (for example
 * L <= 64 with ~10^5 blobs fits; 128^3 does not).  All calls on one GPU
 * share its array: calls that overlap on one GPU (different streams or
 * threads) race and give undefined results. */
#define MB_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
mb_status mb_step_noalloc(const mb_grid_desc* desc, const mb_springs* springs,
                          int64_t nparticles, double* q, void* v, const double* Fext,
                          double* u_out, double* U0_out, double* diag_out,
                          int32_t nsteps, void* stream);

/* Human-readable text for a status. */
const char* mb_status_string(mb_status status);

/* Per-kernel timing (measurement support).  Each launch of a kernel whose
 * id bit is set in kernel_mask (bit i = kernel id i; 0 disables timing)
 * records a pair of HIP events at its own start and end (hipExtLaunchKernel),
 * and the durations are accumulated per kernel id.  mb_grid_kernel_times synchronises the stream, then writes up
 * to `cap` entries of total milliseconds and launch counts per kernel id
 * (ids are stable; names from mb_kernel_name) and returns the number of ids
 * in *n_out.  Setting a mask clears the accumulators. */
mb_status mb_grid_set_timing(mb_grid* grid, uint32_t kernel_mask);

/* Time-stepping scheme of the grid's steps (mb_step, mb_step_ext,
 * mb_step_forced, mb_step_graph); MB_SCHEME_EULER after creation.  The
 * midpoint scheme allocates 6 max_blobs float64 of scratch in the grid at
 * its first step (MB_ERR_NOMEM if that fails) and costs, per step, one more
 * binning and two more interpolations (unsteady), or a second force
 * evaluation, spreading and solve (steady).  u_out then receives the
 * velocity of the update, J(q*)(v^n + v^{n+1})/2 (steady: J(q*) v(q*)), and
 * the diagnostics' sum F the forces at q*.  mb_step_adjoint differentiates
 * the first-order scheme only (MB_ERR_UNSUPPORTED otherwise).
 * MB_ERR_INVALID for an unknown scheme. */
mb_status mb_grid_set_scheme(mb_grid* grid, int32_t scheme);

/* Tiles of the binning, spreading and interpolation: boxes of tx x ty x tz
 * cells, one workgroup each (the binning sorts blobs by tile).  Shapes with
 * kernels: 16x8x8 (the default when 16 divides L, else 8x8x8), 8x8x8,
 * 32x8x8, 16x16x8, 16x8x16, 8x16x16; each extent must divide L
 * (MB_ERR_INVALID otherwise).  Results do not depend on the shape beyond
 * rounding (the fixed-point scale of the spreading is per tile).  The call
 * waits for the device and reallocates the grid's tile scratch
 * (MB_ERR_NOMEM if that fails). */
mb_status mb_grid_set_tiles(mb_grid* grid, int32_t tx, int32_t ty, int32_t tz);
/* The current tile shape into shape_out[3]. */
mb_status mb_grid_get_tiles(const mb_grid* grid, int32_t* shape_out);

/* Tile autotuner: times `nsteps` steps (after one untimed step) of the given
 * state with every tile shape that fits L, on copies of q and v (the
 * caller's q and v are not changed), keeps the fastest shape in the grid
 * and writes it to shape_out[3] (may be NULL).  Arguments as mb_step
 * (nsteps >= 1); synchronises `stream`.  Allocates the copies for the
 * duration of the call (MB_ERR_NOMEM if that fails). */
mb_status mb_grid_autotune(mb_grid* grid, const mb_springs* springs,
                           int64_t nparticles, const double* q, const void* v,
                           const double* Fext, int32_t nsteps, void* stream,
                           int32_t* shape_out);
mb_status mb_grid_kernel_times(mb_grid* grid, void* stream, double* ms_out,
                               int64_t* launches_out, int32_t cap,
                               int32_t* n_out);
const char* mb_kernel_name(int32_t id);

#ifdef __cplusplus
}
#endif
#endif
