/*
 * mbo.h -- the oracle: a plain, slow FP64 CPU implementation of one
 * multiblob immersed-boundary step.  TEST INFRASTRUCTURE ONLY: it exists so
 * that the tests, the smoke check and the CPU baseline of the benchmark can
 * compare the GPU library against an independent computation.  The product
 * path never calls it.  It shares no code, header or table with the GPU
 * library.
 *
 * Notation follows Vazquez-Quesada, Balboa Usabiaga, Delgado-Buscalioni,
 * "A multiblob approach to colloidal hydrodynamics with inherent
 * lubrication" (arXiv:1407.5600):
 *   q_i   blob positions,  F_i blob forces,  h mesh size,
 *   J_i   interpolation (eq. ju),  S_i = J_i^* spreading (Sec. "Multiblob
 *         particle model"),  delta_h the blob kernel (eq. delta),
 *   P     the solenoidal projector, fluid equation eq. vf.
 *
 * Conventions (readings of points the paper leaves open):
 *   - Periodic cubic box of L^3 cells of side h; staggered (MAC) velocity:
 *     component a of node (i,j,k) sits at h*(i,j,k) + (h/2) e_a.
 *   - Fields are stored [3][L][L][L], x fastest.  Positions [M][3].
 *   - Blobs of particle p are 13p .. 13p+12 when blobs_per_particle = 13.
 *
 * Parity status of each function is in the comment above it.
 */
#ifndef MBO_H
#define MBO_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int    L;          /* cells per side */
    double h;          /* mesh size */
    double rho;        /* fluid density (unsteady mode) */
    double eta;        /* dynamic viscosity */
    double dt;         /* time step */
    int    steady;     /* 0: Crank-Nicolson unsteady Stokes; 1: steady Stokes */
    int    zero_mean;  /* 1: the k = 0 mode of the velocity is held at zero */
} mbo_params;

/* 3-point kernel Phi(r), r in units of h (eq. delta; moments stated right
 * after it).  Pinned: partition of unity, zero first moment, sum of squares
 * 1/2, support 3h. */
double mbo_phi(double r);

/* Spreading S: f_a(x) = sum_i delta_h(x - q_i) F_{i,a} at every staggered
 * node (definition of S_i after eq. jm).  f is a force density.  Pinned:
 * adjointness with mbo_interpolate, total force, one-blob J S = 1/(8h^3). */
void mbo_spread(const mbo_params* p, long M, const double* q, const double* F,
                double* f);

/* Interpolation J: u_{i,a} = sum_x h^3 delta_h(x - q_i) v_a(x)  (eq. ju with
 * the integral replaced by the lattice sum).  Pinned: constants and linear
 * fields reproduced exactly, second moment identity (eq. jm2a). */
void mbo_interpolate(const mbo_params* p, long M, const double* q,
                     const double* v, double* u);

/* Harmonic springs inside each particle (Fig. 1 caption, Sec. "Multiblob
 * dynamics"): energy sum (k/2)(|q_b - q_a| - r0)^2 over the pair table,
 * plus Fext of the particle split evenly over its blobs.  Pinned: F = -grad E
 * by finite differences, zero net internal force, zero force at rest. */
void mbo_spring_forces(long P, int nb, int npairs, const int* pa,
                       const int* pb, const double* r0, double k,
                       const double* q, const double* Fext, double* F);

/* 1-D complex DFT, X[m] = sum_j x[j] exp(sign 2 pi i m j / n), computed by
 * recursive mixed-radix Cooley-Tukey.  x is interleaved (re, im), element j
 * at x[2*j*stride].  In place.  Pinned against the direct sum (mbo_dft). */
void mbo_fft(int n, double* x, long stride, int sign);

/* Direct O(n^2) DFT, same convention; used only to pin mbo_fft. */
void mbo_dft(int n, const double* in, double* out, int sign);

/* 3-D complex DFT of an L^3 interleaved complex array, x fastest. */
void mbo_fft3(int L, double* a, int sign);

/* Discrete divergence D (faces to cell centres) of a staggered field:
 * (Dv)_c = sum_b (v_b[c] - v_b[c - e_b]) / h.  out has L^3 entries. */
void mbo_divergence(const mbo_params* p, const double* v, double* out);

/* Fluid solve of eq. vf without the convective and fluctuating stresses
 * (zero Reynolds number, no thermal noise):
 *   unsteady, Crank-Nicolson:
 *     rho (v' - v)/dt = (eta/2) L (v' + v) - G pi + f,   D v' = 0
 *   steady Stokes:  0 = eta L v' - G pi + f,  D v' = 0,  mean(v') = 0
 * solved exactly in Fourier space on the MAC grid.  The k = 0 mode obeys
 * mean(v') = mean(v) + (dt/rho) mean(f) unless zero_mean (or steady).
 * Pinned: dense real-space solve on a tiny grid, D v' = 0, shear-mode decay
 * factor, steady sinusoidal response, momentum balance. */
void mbo_fluid_solve(const mbo_params* p, const double* v_in, const double* f,
                     double* v_out);

/* One or more time steps (scheme: springs at q^n, spread, fluid solve,
 * interpolate the new velocity at q^n, move q by dt*u):
 *   F^n = springs(q^n) + Fext/nb;  f = S(q^n) F^n;  v^{n+1} = solve(v^n, f);
 *   u = J(q^n) v^{n+1};  q^{n+1} = q^n + dt u;  U0_p = mean of u over p.
 * u and U0 (may be NULL) receive the last step's values.  diag (may be NULL)
 * receives {Pi_x, Pi_y, Pi_z, sumF_x, sumF_y, sumF_z, max|Dv|} of the last
 * step, with Pi = rho h^3 sum v after the step and sumF the blob forces of
 * that step.  Parity of long trajectories: unpinned beyond the invariants. */
void mbo_step(const mbo_params* p, long P, int nb, int npairs, const int* pa,
              const int* pb, const double* r0, double k, double* q, double* v,
              const double* Fext, double* u, double* U0, int nsteps,
              double* diag);

/* mbo_step with a force density f_fluid [3][L][L][L] on the fluid (may be
 * NULL) added to S(q^n) F^n in every step: the periodic forcing of the
 * viscosity measurement (Sec. Stresslet and Viscosity). */
void mbo_step_forced(const mbo_params* p, long P, int nb, int npairs,
                     const int* pa, const int* pb, const double* r0, double k,
                     double* q, double* v, const double* Fext,
                     const double* f_fluid, double* u, double* U0, int nsteps,
                     double* diag);

/* Second-order step: a midpoint predictor-corrector rebuilt from eqs. vf,
 * ju and blob1 (m_e = 0), the inertial coupling scheme the paper cites
 * without printing it.  Unsteady: q* = q^n + (dt/2) J(q^n) v^n; v^{n+1} by
 * the Crank-Nicolson solve from v^n with f = S(q*) F(q*); q^{n+1} = q^n +
 * dt J(q*) (v^n + v^{n+1})/2.  Steady: the explicit midpoint rule with two
 * steady solves, at q^n and at q*.  Arguments and outputs as
 * mbo_step_forced. */
void mbo_step_midpoint(const mbo_params* p, long P, int nb, int npairs,
                       const int* pa, const int* pb, const double* r0, double k,
                       double* q, double* v, const double* Fext,
                       const double* f_fluid, double* u, double* U0, int nsteps,
                       double* diag);

/* ---- Derivatives (reverse mode), for the gradient of a trajectory loss.
 * The transposed chain rule of the functions above written out; each is
 * pinned by central finite differences of its forward function. */

/* Phi'(r).  Pinned: finite differences of mbo_phi, sum_j Phi'(x - j) = 0,
 * sum_j (x - j) Phi'(x - j) = -1. */
double mbo_phi_deriv(double r);

/* g_i += sum_a W_{i,a} grad_{q_i} (J_i v)_a: the derivative of the
 * interpolation with respect to the blob positions, contracted with the
 * blob-space weights W [M][3].  Pinned: finite differences of
 * mbo_interpolate. */
void mbo_interpolate_grad(const mbo_params* p, long M, const double* q,
                          const double* v, const double* W, double* g);

/* Transposed Jacobian of the spring forces (without Fext) applied to Fbar
 * [M][3]: qbar += (dF/dq)^T Fbar, *kbar += Fbar . dF/dk, r0bar[e] +=
 * Fbar . dF/dr0_e summed over particles (kbar, r0bar may be NULL).  Pinned:
 * finite differences of mbo_spring_forces. */
void mbo_spring_adjoint(long P, int nb, int npairs, const int* pa,
                        const int* pb, const double* r0, double k,
                        const double* q, const double* Fbar, double* qbar,
                        double* kbar, double* r0bar);

/* Loss of an nsteps trajectory and its gradient.  The step is mbo_step's
 * with per-blob external forces G [M][3] in place of Fext:
 *   F^n = springs(q^n; k, r0) + G;  v^{n+1} = solve(v^n, S(q^n) F^n);
 *   u^n = J(q^n) v^{n+1};  q^{n+1} = q^n + dt u^n.
 * loss = sum_p |U_p - V_p|^2 with U_p the mean of u over particle p's blobs
 * in the last step and V [P][3] the targets.  Returns the loss and its
 * gradients with respect to q^0 [M][3], v^0 [3][L^3], G [M][3], k and the
 * rest lengths r0 [npairs], by the reverse sweep over stored states.
 * Pinned: central finite differences of the forward loss. */
void mbo_loss_grad(const mbo_params* p, long P, int nb, int npairs,
                   const int* pa, const int* pb, const double* r0, double k,
                   const double* q0, const double* v0, const double* G,
                   const double* V, int nsteps, double* loss, double* qbar0,
                   double* vbar0, double* Gbar, double* kbar, double* r0bar);

#ifdef __cplusplus
}
#endif
#endif
