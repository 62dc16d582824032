/*
 * mbo.c -- the oracle (test infrastructure only; see mbo.h).
 *
 * Every routine is the plain definition written out in FP64 with no
 * blocking, fusion or reordering: per-blob loops over kernel supports,
 * a recursive mixed-radix DFT, and an exact Fourier-space solve of the
 * discrete Stokes equations on the staggered grid.
 *
 * Loops whose iterations are independent (blobs of the interpolation,
 * particles of the springs, components of the spreading, lines of the FFT,
 * wavevectors of the solve) carry OpenMP pragmas.  Only the timing build of
 * the CPU baseline enables them; the checker is built without OpenMP and
 * runs every loop serially.  Either build gives the same bits: no iteration
 * reads what another writes, and no sum changes its order.
 */
#include "mbo.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef double complex cplx;

static long wrap_index(long n, long L)
{
    long m = n % L;
    return m < 0 ? m + L : m;
}

/* ------------------------------------------------------------------------
 * Blob kernel.  Phi is the 3-point function of eq. delta.  The paper fixes it
 * through the properties it lists after eq. delta: sum_j Phi(x - j) = 1,
 * sum_j (x - j) Phi(x - j) = 0 and sum_j Phi(x - j)^2 = 1/2 (the discrete L2
 * norm giving int delta_h^2 = 1/(8 h^3)), with a support of three cells.
 * Those conditions determine the function below.
 * ---------------------------------------------------------------------- */
double mbo_phi(double r)
{
    double a = fabs(r);
    if (a <= 0.5)
        return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;
    if (a <= 1.5)
        return (5.0 - 3.0 * a - sqrt(1.0 - 3.0 * (1.0 - a) * (1.0 - a))) / 6.0;
    return 0.0;
}

/* One-dimensional kernel values along axis b for a node set offset by
 * `shift` cells (1/2 along the velocity component's own axis on the MAC
 * grid).  Nodes first .. first+4 bracket the support |r| < 3/2 h.          */
static void axis_weights(double qb, double h, double shift, long* first,
                         double w[5])
{
    long base = (long)floor(qb / h - shift);
    *first = base - 2;
    for (int o = 0; o < 5; ++o) {
        double xnode = ((double)(*first + o) + shift) * h;
        w[o] = mbo_phi((xnode - qb) / h);
    }
}

/* Spreading, S_i F_i = delta_h(r - q_i) F_i (Sec. "Multiblob particle
 * model", definition of S_i as the adjoint of J_i). */
void mbo_spread(const mbo_params* p, long M, const double* q, const double* F,
                double* f)
{
    const long L = p->L;
    const long N = L * L * L;
    const double h = p->h;
    const double inv_vol = 1.0 / (h * h * h);
    memset(f, 0, sizeof(double) * 3 * N);
    /* each component's field takes its contributions in blob order */
#pragma omp parallel for schedule(static)
    for (int a = 0; a < 3; ++a) {
        for (long i = 0; i < M; ++i) {
            long first[3];
            double w[3][5];
            for (int b = 0; b < 3; ++b)
                axis_weights(q[3 * i + b], h, a == b ? 0.5 : 0.0, &first[b],
                             w[b]);
            for (int oz = 0; oz < 5; ++oz)
                for (int oy = 0; oy < 5; ++oy)
                    for (int ox = 0; ox < 5; ++ox) {
                        double delta =
                            inv_vol * w[0][ox] * w[1][oy] * w[2][oz];
                        if (delta == 0.0)
                            continue;
                        long node = wrap_index(first[2] + oz, L) * L * L +
                                    wrap_index(first[1] + oy, L) * L +
                                    wrap_index(first[0] + ox, L);
                        f[a * N + node] += delta * F[3 * i + a];
                    }
        }
    }
}

/* Interpolation, u_i = J_i v = sum over lattice cells of
 * h^3 delta_h(r - q_i) v(r) (eq. ju); the cell volume h^3 cancels the
 * h^-3 of delta_h, leaving the product of the three 1-D weights. */
void mbo_interpolate(const mbo_params* p, long M, const double* q,
                     const double* v, double* u)
{
    const long L = p->L;
    const long N = L * L * L;
    const double h = p->h;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < M; ++i) {
        for (int a = 0; a < 3; ++a) {
            long first[3];
            double w[3][5];
            for (int b = 0; b < 3; ++b)
                axis_weights(q[3 * i + b], h, a == b ? 0.5 : 0.0, &first[b],
                             w[b]);
            double acc = 0.0;
            for (int oz = 0; oz < 5; ++oz)
                for (int oy = 0; oy < 5; ++oy)
                    for (int ox = 0; ox < 5; ++ox) {
                        double weight = w[0][ox] * w[1][oy] * w[2][oz];
                        if (weight == 0.0)
                            continue;
                        long node = wrap_index(first[2] + oz, L) * L * L +
                                    wrap_index(first[1] + oy, L) * L +
                                    wrap_index(first[0] + ox, L);
                        acc += weight * v[a * N + node];
                    }
            u[3 * i + a] = acc;
        }
    }
}

/* Harmonic springs between blob pairs of each particle (Fig. 1: hard springs
 * holding the blobs at the icosahedron sites).  With d = q_b - q_a the force
 * on blob a is +k (|d| - r0) d/|d| and on blob b its negative. */
void mbo_spring_forces(long P, int nb, int npairs, const int* pa,
                       const int* pb, const double* r0, double k,
                       const double* q, const double* Fext, double* F)
{
#pragma omp parallel for schedule(static)
    for (long p = 0; p < P; ++p) {
        for (int b = 0; b < nb; ++b)
            for (int c = 0; c < 3; ++c)
                F[3 * (p * nb + b) + c] = Fext ? Fext[3 * p + c] / nb : 0.0;
        for (int e = 0; e < npairs; ++e) {
            long ia = p * nb + pa[e];
            long ib = p * nb + pb[e];
            double d[3];
            double len2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                d[c] = q[3 * ib + c] - q[3 * ia + c];
                len2 += d[c] * d[c];
            }
            double len = sqrt(len2);
            double s = k * (len - r0[e]) / len;
            for (int c = 0; c < 3; ++c) {
                F[3 * ia + c] += s * d[c];
                F[3 * ib + c] -= s * d[c];
            }
        }
    }
}

/* ------------------------------------------------------------------------
 * Discrete Fourier transform.
 * ---------------------------------------------------------------------- */
static int smallest_factor(int n)
{
    for (int f = 2; f * f <= n; ++f)
        if (n % f == 0)
            return f;
    return n;
}

/* Recursive decimation in time.  Input element j is in[j * istride]; the n
 * outputs go to out[0 .. n-1].  W[k] = exp(sign 2 pi i k / n0) with n | n0. */
static void fft_rec(int n, const cplx* in, long istride, cplx* out,
                    const cplx* W, int n0)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    int pf = smallest_factor(n);
    int m = n / pf;
    for (int r = 0; r < pf; ++r)
        fft_rec(m, in + r * istride, istride * pf, out + r * m, W, n0);
    cplx* tmp = (cplx*)malloc(sizeof(cplx) * n);
    long step = n0 / n;
    for (int s = 0; s < pf; ++s)
        for (int kk = 0; kk < m; ++kk) {
            long K = kk + (long)s * m;
            cplx acc = 0.0;
            for (int r = 0; r < pf; ++r)
                acc += W[((long)r * K % n) * step] * out[r * m + kk];
            tmp[K] = acc;
        }
    memcpy(out, tmp, sizeof(cplx) * n);
    free(tmp);
}

static cplx* twiddle_table(int n, int sign)
{
    cplx* W = (cplx*)malloc(sizeof(cplx) * n);
    for (int k = 0; k < n; ++k) {
        double ang = 2.0 * M_PI * (double)k / (double)n;
        W[k] = cos(ang) + I * (sign * sin(ang));
    }
    return W;
}

/* One line, with a prebuilt table. */
static void fft_line(int n, cplx* x, long stride, const cplx* W, cplx* in,
                     cplx* out)
{
    for (int j = 0; j < n; ++j)
        in[j] = x[j * stride];
    fft_rec(n, in, 1, out, W, n);
    for (int j = 0; j < n; ++j)
        x[j * stride] = out[j];
}

void mbo_fft(int n, double* x, long stride, int sign)
{
    cplx* W = twiddle_table(n, sign);
    cplx* in = (cplx*)malloc(sizeof(cplx) * n);
    cplx* out = (cplx*)malloc(sizeof(cplx) * n);
    fft_line(n, (cplx*)x, stride, W, in, out);
    free(W);
    free(in);
    free(out);
}

void mbo_dft(int n, const double* in_, double* out_, int sign)
{
    const cplx* in = (const cplx*)in_;
    cplx* out = (cplx*)out_;
    for (int m = 0; m < n; ++m) {
        cplx acc = 0.0;
        for (int j = 0; j < n; ++j) {
            double ang = 2.0 * M_PI * (double)(((long)m * j) % n) / (double)n;
            acc += in[j] * (cos(ang) + I * (sign * sin(ang)));
        }
        out[m] = acc;
    }
}

void mbo_fft3(int L, double* a_, int sign)
{
    cplx* a = (cplx*)a_;
    cplx* W = twiddle_table(L, sign);
    long LL = (long)L * L;
    /* the lines of one direction are independent of one another */
#pragma omp parallel
    {
        cplx* in = (cplx*)malloc(sizeof(cplx) * L);
        cplx* out = (cplx*)malloc(sizeof(cplx) * L);
#pragma omp for schedule(static)
        for (long z = 0; z < L; ++z) /* along x */
            for (long y = 0; y < L; ++y)
                fft_line(L, a + z * LL + y * L, 1, W, in, out);
#pragma omp for schedule(static)
        for (long z = 0; z < L; ++z) /* along y */
            for (long x = 0; x < L; ++x)
                fft_line(L, a + z * LL + x, L, W, in, out);
#pragma omp for schedule(static)
        for (long y = 0; y < L; ++y) /* along z */
            for (long x = 0; x < L; ++x)
                fft_line(L, a + y * L + x, LL, W, in, out);
        free(in);
        free(out);
    }
    free(W);
}

/* ------------------------------------------------------------------------
 * Staggered-grid operators and the fluid solve.
 * ---------------------------------------------------------------------- */
void mbo_divergence(const mbo_params* p, const double* v, double* out)
{
    const long L = p->L;
    const long N = L * L * L;
    for (long z = 0; z < L; ++z)
        for (long y = 0; y < L; ++y)
            for (long x = 0; x < L; ++x) {
                long c = (z * L + y) * L + x;
                long cx = (z * L + y) * L + wrap_index(x - 1, L);
                long cy = (z * L + wrap_index(y - 1, L)) * L + x;
                long cz = (wrap_index(z - 1, L) * L + y) * L + x;
                out[c] = ((v[c] - v[cx]) + (v[N + c] - v[N + cy]) +
                          (v[2 * N + c] - v[2 * N + cz])) /
                         p->h;
            }
}

/* Exact solve of the discrete equations in Fourier space.  With the forward
 * transform X[m] = sum_j x_j exp(-2 pi i m j / L), the divergence D has the
 * symbol Dh_b = (1 - exp(-2 pi i m_b / L)) / h, the gradient G = -D^T has
 * -conj(Dh), the Laplacian L = D G acts on every velocity component with
 * -|Dh|^2, and the projector onto discretely divergence-free fields is
 * P = 1 - conj(Dh) Dh^T / |Dh|^2 (the operator P of eq. vf). */
void mbo_fluid_solve(const mbo_params* p, const double* v_in, const double* f,
                     double* v_out)
{
    const long L = p->L;
    const long N = L * L * L;
    const double h = p->h;
    cplx* A = (cplx*)malloc(sizeof(cplx) * 3 * N);
    cplx* B = (cplx*)malloc(sizeof(cplx) * 3 * N);
    double vbar[3], fbar[3];
    for (int c = 0; c < 3; ++c) {
        double sv = 0.0, sf = 0.0;
        for (long j = 0; j < N; ++j) {
            A[c * N + j] = v_in[c * N + j];
            B[c * N + j] = f[c * N + j];
            sv += v_in[c * N + j];
            sf += f[c * N + j];
        }
        vbar[c] = sv / (double)N;
        fbar[c] = sf / (double)N;
        mbo_fft3((int)L, (double*)(A + c * N), -1);
        mbo_fft3((int)L, (double*)(B + c * N), -1);
    }
    cplx* Dh = (cplx*)malloc(sizeof(cplx) * L);
    for (long m = 0; m < L; ++m) {
        double ang = 2.0 * M_PI * (double)m / (double)L;
        Dh[m] = (1.0 - (cos(ang) - I * sin(ang))) / h;
    }
#pragma omp parallel for schedule(static)
    for (long mz = 0; mz < L; ++mz)
        for (long my = 0; my < L; ++my)
            for (long mx = 0; mx < L; ++mx) {
                long j = (mz * L + my) * L + mx;
                if (mx == 0 && my == 0 && mz == 0) {
                    for (int c = 0; c < 3; ++c) {
                        double mean = 0.0;
                        if (!p->steady && !p->zero_mean)
                            mean = vbar[c] + p->dt / p->rho * fbar[c];
                        A[c * N + j] = (double)N * mean;
                    }
                    continue;
                }
                cplx D[3] = {Dh[mx], Dh[my], Dh[mz]};
                double D2 = 0.0;
                for (int c = 0; c < 3; ++c)
                    D2 += creal(D[c] * conj(D[c]));
                cplx rhs[3];
                double denom;
                if (p->steady) {
                    for (int c = 0; c < 3; ++c)
                        rhs[c] = B[c * N + j];
                    denom = p->eta * D2;
                } else {
                    double a = p->rho / p->dt - 0.5 * p->eta * D2;
                    for (int c = 0; c < 3; ++c)
                        rhs[c] = a * A[c * N + j] + B[c * N + j];
                    denom = p->rho / p->dt + 0.5 * p->eta * D2;
                }
                cplx div = 0.0;
                for (int c = 0; c < 3; ++c)
                    div += D[c] * rhs[c];
                for (int c = 0; c < 3; ++c)
                    A[c * N + j] = (rhs[c] - conj(D[c]) * div / D2) / denom;
            }
    for (int c = 0; c < 3; ++c) {
        mbo_fft3((int)L, (double*)(A + c * N), +1);
        for (long j = 0; j < N; ++j)
            v_out[c * N + j] = creal(A[c * N + j]) / (double)N;
    }
    free(Dh);
    free(A);
    free(B);
}

/* ------------------------------------------------------------------------
 * Time step.
 * ---------------------------------------------------------------------- */
static void step_outputs(const mbo_params* p, long P, int nb, const double* uu,
                         const double* F, const double* v, double* u, double* U0,
                         double* diag);

void mbo_step(const mbo_params* p, long P, int nb, int npairs, const int* pa,
              const int* pb, const double* r0, double k, double* q, double* v,
              const double* Fext, double* u, double* U0, int nsteps,
              double* diag)
{
    mbo_step_forced(p, P, nb, npairs, pa, pb, r0, k, q, v, Fext, NULL, u, U0,
                    nsteps, diag);
}

/* The step with a force density f_fluid [3][L][L][L] acting on the fluid
 * (NULL: none) added to the spread blob forces before the solve: the
 * periodic forcing f0 sin(k_j y) x of the viscosity measurement (Sec.
 * Stresslet and Viscosity) enters the momentum equation (eq. vf) as a body
 * force density on the fluid. */
void mbo_step_forced(const mbo_params* p, long P, int nb, int npairs,
                     const int* pa, const int* pb, const double* r0, double k,
                     double* q, double* v, const double* Fext,
                     const double* f_fluid, double* u, double* U0, int nsteps,
                     double* diag)
{
    const long L = p->L;
    const long N = L * L * L;
    const long M = P * nb;
    double* F = (double*)malloc(sizeof(double) * 3 * (M > 0 ? M : 1));
    double* uu = (double*)malloc(sizeof(double) * 3 * (M > 0 ? M : 1));
    double* f = (double*)malloc(sizeof(double) * 3 * N);
    for (int n = 0; n < nsteps; ++n) {
        mbo_spring_forces(P, nb, npairs, pa, pb, r0, k, q, Fext, F);
        mbo_spread(p, M, q, F, f);
        if (f_fluid)
            for (long j = 0; j < 3 * N; ++j)
                f[j] += f_fluid[j];
        mbo_fluid_solve(p, v, f, v);
        mbo_interpolate(p, M, q, v, uu);
        for (long i = 0; i < 3 * M; ++i)
            q[i] += p->dt * uu[i];
    }
    if (nsteps > 0)
        step_outputs(p, P, nb, uu, F, v, u, U0, diag);
    free(F);
    free(uu);
    free(f);
}

/* Outputs of the last step: blob velocities u, particle means U0 and the
 * diagnostics (momentum rho h^3 sum v, sum of the blob forces F, max |D v|). */
static void step_outputs(const mbo_params* p, long P, int nb, const double* uu,
                         const double* F, const double* v, double* u, double* U0,
                         double* diag)
{
    const long L = p->L;
    const long N = L * L * L;
    const long M = P * nb;
    if (u)
        memcpy(u, uu, sizeof(double) * 3 * M);
    if (U0)
        for (long pp = 0; pp < P; ++pp)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int b = 0; b < nb; ++b)
                    s += uu[3 * (pp * nb + b) + c];
                U0[3 * pp + c] = s / nb;
            }
    if (diag) {
        double h3 = p->h * p->h * p->h;
        for (int c = 0; c < 3; ++c) {
            double sv = 0.0, sF = 0.0;
            for (long j = 0; j < N; ++j)
                sv += v[c * N + j];
            for (long i = 0; i < M; ++i)
                sF += F[3 * i + c];
            diag[c] = p->rho * h3 * sv;
            diag[3 + c] = sF;
        }
        double* dv = (double*)malloc(sizeof(double) * N);
        mbo_divergence(p, v, dv);
        double mx = 0.0;
        for (long j = 0; j < N; ++j)
            if (fabs(dv[j]) > mx)
                mx = fabs(dv[j]);
        diag[6] = mx;
        free(dv);
    }
}

/* Second-order step: a midpoint predictor-corrector rebuilt from eqs. vf,
 * ju and blob1 with neutrally buoyant blobs (m_e = 0, so the blob-fluid
 * force is minus the blob force), as the inertial coupling scheme the paper
 * uses is cited but not printed.
 *   unsteady:  q* = q^n + (dt/2) J(q^n) v^n
 *              v^{n+1} = CN solve of eq. vf from v^n with f = S(q*) F(q*)
 *              q^{n+1} = q^n + dt J(q*) (v^n + v^{n+1}) / 2
 *   steady:    q* = q^n + (dt/2) J(q^n) v(q^n),  q^{n+1} = q^n + dt J(q*) v(q*)
 *              with v(q) the steady solve of f = S(q) F(q)
 * (f_fluid, may be NULL, is added to f in every solve).  The force and the
 * interpolation are taken at the midpoint and the velocity is the
 * trapezoidal mean, so the step is second order in dt where the
 * first-order step takes both at q^n.  u reports the velocity of the last
 * update, J(q*)(v^n + v^{n+1})/2 (steady: J(q*) v(q*)); the diagnostics'
 * sum F is that of the forces at q*. */
void mbo_step_midpoint(const mbo_params* p, long P, int nb, int npairs,
                       const int* pa, const int* pb, const double* r0, double k,
                       double* q, double* v, const double* Fext,
                       const double* f_fluid, double* u, double* U0, int nsteps,
                       double* diag)
{
    const long L = p->L;
    const long N = L * L * L;
    const long M = P * nb;
    const long m3 = 3 * (M > 0 ? M : 1);
    double* F = (double*)malloc(sizeof(double) * m3);
    double* uu = (double*)malloc(sizeof(double) * m3);
    double* ua = (double*)malloc(sizeof(double) * m3);
    double* qs = (double*)malloc(sizeof(double) * m3);
    double* f = (double*)malloc(sizeof(double) * 3 * N);
    double* vn = (double*)malloc(sizeof(double) * 3 * N);
    const double dt = p->dt;
    for (int n = 0; n < nsteps; ++n) {
        if (!p->steady) {
            mbo_interpolate(p, M, q, v, ua);
        } else {
            mbo_spring_forces(P, nb, npairs, pa, pb, r0, k, q, Fext, F);
            mbo_spread(p, M, q, F, f);
            if (f_fluid)
                for (long j = 0; j < 3 * N; ++j)
                    f[j] += f_fluid[j];
            mbo_fluid_solve(p, v, f, v);
            mbo_interpolate(p, M, q, v, ua);
        }
        for (long i = 0; i < 3 * M; ++i)
            qs[i] = q[i] + 0.5 * dt * ua[i];
        mbo_spring_forces(P, nb, npairs, pa, pb, r0, k, qs, Fext, F);
        mbo_spread(p, M, qs, F, f);
        if (f_fluid)
            for (long j = 0; j < 3 * N; ++j)
                f[j] += f_fluid[j];
        memcpy(vn, v, sizeof(double) * 3 * N);
        mbo_fluid_solve(p, v, f, v);
        if (!p->steady)
            for (long j = 0; j < 3 * N; ++j)
                vn[j] = 0.5 * (vn[j] + v[j]);
        mbo_interpolate(p, M, qs, p->steady ? v : vn, uu);
        for (long i = 0; i < 3 * M; ++i)
            q[i] += dt * uu[i];
    }
    if (nsteps > 0)
        step_outputs(p, P, nb, uu, F, v, u, U0, diag);
    free(F);
    free(uu);
    free(ua);
    free(qs);
    free(f);
    free(vn);
}

/* ------------------------------------------------------------------------
 * Derivatives (reverse mode) of the step.
 *
 * These are the plain transposed chain rule of the functions above, for
 * the gradient of a trajectory loss.  Each is pinned by central finite
 * differences of the corresponding forward function.
 * ---------------------------------------------------------------------- */

/* d Phi / dr of the 3-point kernel (C^1: Phi' is continuous at |r| = 1/2
 * and vanishes at |r| = 3/2). */
double mbo_phi_deriv(double r)
{
    double a = fabs(r);
    double sgn = r < 0.0 ? -1.0 : 1.0;
    if (a <= 0.5)
        return -r / sqrt(1.0 - 3.0 * r * r);
    if (a <= 1.5) {
        double c = 1.0 - a;
        return sgn * (-0.5 - c / (2.0 * sqrt(1.0 - 3.0 * c * c)));
    }
    return 0.0;
}

/* One-dimensional kernel values and their derivatives with respect to the
 * blob coordinate qb (d/dqb Phi((x - qb)/h) = -Phi'((x - qb)/h)/h). */
static void axis_weights_deriv(double qb, double h, double shift, long* first,
                               double w[5], double dw[5])
{
    long base = (long)floor(qb / h - shift);
    *first = base - 2;
    for (int o = 0; o < 5; ++o) {
        double xnode = ((double)(*first + o) + shift) * h;
        double r = (xnode - qb) / h;
        w[o] = mbo_phi(r);
        dw[o] = -mbo_phi_deriv(r) / h;
    }
}

void mbo_interpolate_grad(const mbo_params* p, long M, const double* q,
                          const double* v, const double* W, double* g)
{
    const long L = p->L;
    const long N = L * L * L;
    const double h = p->h;
    for (long i = 0; i < M; ++i) {
        for (int a = 0; a < 3; ++a) {
            long first[3];
            double w[3][5], dw[3][5];
            for (int b = 0; b < 3; ++b)
                axis_weights_deriv(q[3 * i + b], h, a == b ? 0.5 : 0.0,
                                   &first[b], w[b], dw[b]);
            double grad[3] = {0.0, 0.0, 0.0};
            for (int oz = 0; oz < 5; ++oz)
                for (int oy = 0; oy < 5; ++oy)
                    for (int ox = 0; ox < 5; ++ox) {
                        long node = wrap_index(first[2] + oz, L) * L * L +
                                    wrap_index(first[1] + oy, L) * L +
                                    wrap_index(first[0] + ox, L);
                        double val = v[a * N + node];
                        grad[0] += dw[0][ox] * w[1][oy] * w[2][oz] * val;
                        grad[1] += w[0][ox] * dw[1][oy] * w[2][oz] * val;
                        grad[2] += w[0][ox] * w[1][oy] * dw[2][oz] * val;
                    }
            for (int b = 0; b < 3; ++b)
                g[3 * i + b] += W[3 * i + a] * grad[b];
        }
    }
}

void mbo_spring_adjoint(long P, int nb, int npairs, const int* pa,
                        const int* pb, const double* r0, double k,
                        const double* q, const double* Fbar, double* qbar,
                        double* kbar, double* r0bar)
{
    for (long p = 0; p < P; ++p) {
        for (int e = 0; e < npairs; ++e) {
            long ia = p * nb + pa[e];
            long ib = p * nb + pb[e];
            double d[3], lam[3];
            double len2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                d[c] = q[3 * ib + c] - q[3 * ia + c];
                len2 += d[c] * d[c];
                /* the pair force enters F_a with + and F_b with - */
                lam[c] = Fbar[3 * ia + c] - Fbar[3 * ib + c];
            }
            double len = sqrt(len2);
            /* force on a: f = k (1 - r0/|d|) d;
             * df/dd = k [(1 - r0/|d|) I + r0 d d^T / |d|^3] (symmetric) */
            double s = k * (1.0 - r0[e] / len);
            double t = k * r0[e] / (len * len * len);
            double ld = lam[0] * d[0] + lam[1] * d[1] + lam[2] * d[2];
            for (int c = 0; c < 3; ++c) {
                double jl = s * lam[c] + t * d[c] * ld; /* (df/dd)^T lam */
                qbar[3 * ib + c] += jl;                 /* dd/dq_b = +I */
                qbar[3 * ia + c] -= jl;                 /* dd/dq_a = -I */
            }
            if (kbar)
                *kbar += ld * (1.0 - r0[e] / len);      /* df/dk = f/k */
            if (r0bar)
                r0bar[e] += -k * ld / len;              /* df/dr0 = -k d/|d| */
        }
    }
}

/* Apply C = (rho/dt) I + (eta/2) L_h (the explicit half of the
 * Crank-Nicolson step; the 7-point Laplacian per component) to a field. */
static void apply_cn_explicit(const mbo_params* p, const double* x, double* y)
{
    const long L = p->L;
    const long N = L * L * L;
    const double a = p->rho / p->dt;
    const double b = 0.5 * p->eta / (p->h * p->h);
    for (int c = 0; c < 3; ++c)
        for (long z = 0; z < L; ++z)
            for (long yy = 0; yy < L; ++yy)
                for (long xx = 0; xx < L; ++xx) {
                    const double* X = x + c * N;
                    long idx = (z * L + yy) * L + xx;
                    double lap = X[(z * L + yy) * L + wrap_index(xx - 1, L)] +
                                 X[(z * L + yy) * L + wrap_index(xx + 1, L)] +
                                 X[(z * L + wrap_index(yy - 1, L)) * L + xx] +
                                 X[(z * L + wrap_index(yy + 1, L)) * L + xx] +
                                 X[(wrap_index(z - 1, L) * L + yy) * L + xx] +
                                 X[(wrap_index(z + 1, L) * L + yy) * L + xx] -
                                 6.0 * X[idx];
                    y[c * N + idx] = a * X[idx] + b * lap;
                }
}

void mbo_loss_grad(const mbo_params* p, long P, int nb, int npairs,
                   const int* pa, const int* pb, const double* r0, double k,
                   const double* q0, const double* v0, const double* G,
                   const double* V, int nsteps, double* loss, double* qbar0,
                   double* vbar0, double* Gbar, double* kbar, double* r0bar)
{
    const long L = p->L;
    const long N = L * L * L;
    const long M = P * nb;
    const double h3 = p->h * p->h * p->h;
    const long MM = M > 0 ? M : 1;
    /* forward, keeping q^n and v^{n+1} of every step */
    double* qs = (double*)malloc(sizeof(double) * 3 * MM * (nsteps + 1));
    double* vs = (double*)malloc(sizeof(double) * 3 * N * (nsteps + 1));
    double* F = (double*)malloc(sizeof(double) * 3 * MM);
    double* f = (double*)malloc(sizeof(double) * 3 * N);
    double* u = (double*)malloc(sizeof(double) * 3 * MM);
    memcpy(qs, q0, sizeof(double) * 3 * M);
    memcpy(vs, v0, sizeof(double) * 3 * N);
    for (int n = 0; n < nsteps; ++n) {
        double* q = qs + 3 * M * n;
        mbo_spring_forces(P, nb, npairs, pa, pb, r0, k, q, NULL, F);
        for (long i = 0; i < 3 * M; ++i)
            F[i] += G[i];
        mbo_spread(p, M, q, F, f);
        mbo_fluid_solve(p, vs + 3 * N * n, f, vs + 3 * N * (n + 1));
        mbo_interpolate(p, M, q, vs + 3 * N * (n + 1), u);
        for (long i = 0; i < 3 * M; ++i)
            qs[3 * M * (n + 1) + i] = q[i] + p->dt * u[i];
    }
    /* loss = sum_p |U_p - V_p|^2 with U_p the mean blob velocity of the last
     * step; dloss/du_i = 2 (U_p - V_p) / nb */
    double* ubar = (double*)calloc(3 * MM, sizeof(double));
    double l = 0.0;
    if (nsteps > 0) {
        for (long pp = 0; pp < P; ++pp)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int b = 0; b < nb; ++b)
                    s += u[3 * (pp * nb + b) + c];
                double dU = s / nb - V[3 * pp + c];
                l += dU * dU;
                for (int b = 0; b < nb; ++b)
                    ubar[3 * (pp * nb + b) + c] = 2.0 * dU / nb;
            }
    }
    *loss = l;
    /* reverse sweep */
    double* qbar = (double*)calloc(3 * MM, sizeof(double));
    double* vbar = (double*)calloc(3 * N, sizeof(double));
    double* wbar = (double*)malloc(sizeof(double) * 3 * N);
    double* fbar = (double*)malloc(sizeof(double) * 3 * N);
    double* zero = (double*)calloc(3 * N, sizeof(double));
    double* Fbar = (double*)malloc(sizeof(double) * 3 * MM);
    double* Wt = (double*)malloc(sizeof(double) * 3 * MM);
    for (long i = 0; i < 3 * M; ++i)
        Gbar[i] = 0.0;
    *kbar = 0.0;
    for (int e = 0; e < npairs; ++e)
        r0bar[e] = 0.0;
    for (int n = nsteps - 1; n >= 0; --n) {
        const double* q = qs + 3 * M * n;
        const double* vn1 = vs + 3 * N * (n + 1);
        /* q^{n+1} = q^n + dt u^n */
        for (long i = 0; i < 3 * M; ++i)
            ubar[i] += p->dt * qbar[i];
        /* u^n = J(q^n) v^{n+1}: position part, and J^T = h^3 S */
        mbo_interpolate_grad(p, M, q, vn1, ubar, qbar);
        for (long i = 0; i < 3 * M; ++i)
            Wt[i] = h3 * ubar[i];
        mbo_spread(p, M, q, Wt, wbar);
        for (long j = 0; j < 3 * N; ++j)
            wbar[j] += vbar[j];
        /* v^{n+1} = Q (C v^n + f^n) with Q = P K^-1 symmetric and commuting
         * with C: fbar = Q wbar, vbar = C Q wbar.  Q is the fluid solve with
         * a zero input velocity (steady: the whole solve). */
        mbo_fluid_solve(p, zero, wbar, fbar);
        if (p->steady)
            memset(vbar, 0, sizeof(double) * 3 * N);
        else
            apply_cn_explicit(p, fbar, vbar);
        /* f^n = S(q^n) F^n: F part (S^T = h^-3 J) and position part */
        mbo_spring_forces(P, nb, npairs, pa, pb, r0, k, q, NULL, F);
        for (long i = 0; i < 3 * M; ++i)
            F[i] += G[i];
        mbo_interpolate(p, M, q, fbar, Fbar);
        for (long i = 0; i < 3 * M; ++i) {
            Fbar[i] /= h3;
            Wt[i] = F[i] / h3;
        }
        mbo_interpolate_grad(p, M, q, fbar, Wt, qbar);
        /* F^n = springs(q^n; k, r0) + G */
        mbo_spring_adjoint(P, nb, npairs, pa, pb, r0, k, q, Fbar, qbar, kbar,
                           r0bar);
        for (long i = 0; i < 3 * M; ++i) {
            Gbar[i] += Fbar[i];
            ubar[i] = 0.0;
        }
    }
    memcpy(qbar0, qbar, sizeof(double) * 3 * M);
    memcpy(vbar0, vbar, sizeof(double) * 3 * N);
    free(qs); free(vs); free(F); free(f); free(u); free(ubar); free(qbar);
    free(vbar); free(wbar); free(fbar); free(zero); free(Fbar); free(Wt);
}

