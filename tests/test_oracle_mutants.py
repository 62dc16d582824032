"""Planted mistakes: each mutation below is applied to a copy of the
oracle's C source, compiled on the CPU, and the oracle's pin tests are run
against it in a subprocess; every mutant must fail at least one pin.  This
shows that the pins tie down every part of the oracle (kernel, staggering,
spreading, interpolation, springs, DFT, projection, Crank-Nicolson, mean
mode, derivatives, fluid forcing, the second-order step)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mbo.c")
PINS = ["tests/test_oracle_kernel.py", "tests/test_oracle_fft.py",
        "tests/test_oracle_operators.py", "tests/test_oracle_springs.py",
        "tests/test_oracle_solver.py", "tests/test_oracle_step.py",
        "tests/test_oracle_adjoint.py", "tests/test_oracle_stokes.py",
        "tests/test_oracle_midpoint.py"]

MUTANTS = {
    "kernel_sqrt_sign": ("return (1.0 + sqrt(1.0 - 3.0 * a * a)) / 3.0;",
                         "return (1.0 - sqrt(1.0 - 3.0 * a * a)) / 3.0;"),
    "kernel_outer_branch": ("return (5.0 - 3.0 * a - sqrt(",
                            "return (5.0 - 3.0 * a + sqrt("),
    # first occurrence: the staggering shift inside the spreading loop only
    "stagger_shift_sign": ("a == b ? 0.5 : 0.0", "a == b ? -0.5 : 0.0"),
    "spread_no_volume": ("inv_vol * w[0][ox] * w[1][oy] * w[2][oz];",
                         "w[0][ox] * w[1][oy] * w[2][oz];"),
    "interp_transposed_axes": ("double weight = w[0][ox] * w[1][oy] * w[2][oz];",
                               "double weight = w[0][oz] * w[1][oy] * w[2][ox];"),
    "spring_sign": ("F[3 * ia + c] += s * d[c];", "F[3 * ia + c] -= s * d[c];"),
    "spring_rest_length": ("double s = k * (len - r0[e]) / len;",
                           "double s = k * (len - r0[e]);"),
    "fft_twiddle_stride": ("acc += W[((long)r * K % n) * step] * out[r * m + kk];",
                           "acc += W[((long)r * K % n)] * out[r * m + kk];"),
    "symbol_sign": ("Dh[m] = (1.0 - (cos(ang) - I * sin(ang))) / h;",
                    "Dh[m] = (1.0 - (cos(ang) + I * sin(ang))) / h;"),
    "projector_no_conj": ("A[c * N + j] = (rhs[c] - conj(D[c]) * div / D2) / denom;",
                          "A[c * N + j] = (rhs[c] - D[c] * div / D2) / denom;"),
    "projector_sign": ("A[c * N + j] = (rhs[c] - conj(D[c]) * div / D2) / denom;",
                       "A[c * N + j] = (rhs[c] + conj(D[c]) * div / D2) / denom;"),
    "cn_explicit_half": ("double a = p->rho / p->dt - 0.5 * p->eta * D2;",
                         "double a = p->rho / p->dt - p->eta * D2;"),
    "cn_implicit_half": ("denom = p->rho / p->dt + 0.5 * p->eta * D2;",
                         "denom = p->rho / p->dt + p->eta * D2;"),
    "mean_mode_density": ("mean = vbar[c] + p->dt / p->rho * fbar[c];",
                          "mean = vbar[c] + p->dt * fbar[c];"),
    "steady_viscosity": ("denom = p->eta * D2;", "denom = D2;"),
    "divergence_index": ("long cy = (z * L + wrap_index(y - 1, L)) * L + x;",
                         "long cy = (z * L + wrap_index(y + 1, L)) * L + x;"),
    # reverse-mode derivatives
    "phi_deriv_inner": ("return -r / sqrt(1.0 - 3.0 * r * r);",
                        "return r / sqrt(1.0 - 3.0 * r * r);"),
    "interp_grad_axis": ("grad[1] += w[0][ox] * dw[1][oy] * w[2][oz] * val;",
                         "grad[1] += w[0][ox] * w[1][oy] * dw[2][oz] * val;"),
    "spring_jacobian_drop_dd": ("double jl = s * lam[c] + t * d[c] * ld;",
                                "double jl = s * lam[c];"),
    "adjoint_position_update": ("ubar[i] += p->dt * qbar[i];", "ubar[i] += qbar[i];"),
    "adjoint_transpose_volume": ("Wt[i] = h3 * ubar[i];", "Wt[i] = ubar[i];"),
    "adjoint_cn_explicit": ("y[c * N + idx] = a * X[idx] + b * lap;",
                            "y[c * N + idx] = a * X[idx] - b * lap;"),
    # fluid forcing and the second-order step
    "forced_drop_fluid_force": ("f[j] += f_fluid[j];", "f[j] += 0.0 * f_fluid[j];"),
    "midpoint_predictor_full_step": ("qs[i] = q[i] + 0.5 * dt * ua[i];",
                                     "qs[i] = q[i] + dt * ua[i];"),
    "midpoint_forces_at_start": ("mbo_spring_forces(P, nb, npairs, pa, pb, r0, k, qs, Fext, F);",
                                 "mbo_spring_forces(P, nb, npairs, pa, pb, r0, k, q, Fext, F);"),
    "midpoint_no_trapezoid": ("vn[j] = 0.5 * (vn[j] + v[j]);", "vn[j] = v[j];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    c_path = tmp_path / "mbo.c"
    c_path.write_text(mutated)
    import shutil
    shutil.copy(os.path.join(ROOT, "oracle", "mbo.h"), tmp_path / "mbo.h")
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(lib),
                    str(c_path), "-lm"], check=True)
    env = dict(os.environ, MBO_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"
