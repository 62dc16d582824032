/*
 * mbo.c -- the oracle (test infrastructure only; see mbo.h).
 *
 * Every routine is the plain definition written out in FP64 with no
 * blocking, fusion or reordering: per-blob loops over kernel supports,
 * a recursive mixed-radix DFT, and an exact Fourier-space solve of the
 * discrete Stokes equations on the staggered grid.
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
    for (long i = 0; i < M; ++i) {
        for (int a = 0; a < 3; ++a) {
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
    cplx* in = (cplx*)malloc(sizeof(cplx) * L);
    cplx* out = (cplx*)malloc(sizeof(cplx) * L);
    long LL = (long)L * L;
    for (long z = 0; z < L; ++z) /* along x */
        for (long y = 0; y < L; ++y)
            fft_line(L, a + z * LL + y * L, 1, W, in, out);
    for (long z = 0; z < L; ++z) /* along y */
        for (long x = 0; x < L; ++x)
            fft_line(L, a + z * LL + x, L, W, in, out);
    for (long y = 0; y < L; ++y) /* along z */
        for (long x = 0; x < L; ++x)
            fft_line(L, a + y * L + x, LL, W, in, out);
    free(W);
    free(in);
    free(out);
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
void mbo_step(const mbo_params* p, long P, int nb, int npairs, const int* pa,
              const int* pb, const double* r0, double k, double* q, double* v,
              const double* Fext, double* u, double* U0, int nsteps,
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
        mbo_fluid_solve(p, v, f, v);
        mbo_interpolate(p, M, q, v, uu);
        for (long i = 0; i < 3 * M; ++i)
            q[i] += p->dt * uu[i];
    }
    if (nsteps > 0) {
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
    free(F);
    free(uu);
    free(f);
}
