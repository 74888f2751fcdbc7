"""Each plausible slip in the oracle must fail at least one pin.

Every case copies the oracle's C source, plants one mistake (a dropped term, a
flipped sign, a transposed index, a wrong constant), builds it with the same
flags and runs the pin suite against that build in a fresh process.  The pin
suite must fail for every mutant.  Nothing is planted in the real oracle.
"""
import concurrent.futures
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_vans_oracle.c")

MUTANTS = {
    "feq_linear_sign": ("1.0 + eu / CS2", "1.0 - eu / CS2"),
    "feq_drop_uu": ("- uu / (2.0 * CS2))", ")"),
    "feq_quadratic_coeff": ("(eu * eu) / (2.0 * CS2 * CS2)", "(eu * eu) / (2.0 * CS2)"),
    "source_sign_u": ("double cx = (EX[i] - ux) / CS2", "double cx = (EX[i] + ux) / CS2"),
    "source_drop_prefactor": ("double pre = 1.0 - 1.0 / (2.0 * tau);", "double pre = 1.0;"),
    "source_drop_second_order": ("+ eu * EX[i] / (CS2 * CS2)", ""),
    "ergun_darcy_constant": ("/ (150.0 * (1.0 - eps) * (1.0 - eps))", "/ (180.0 * (1.0 - eps) * (1.0 - eps))"),
    "ergun_forchheimer_constant": ("Feps = 1.75 / sqrt", "Feps = 1.5 / sqrt"),
    "darcy_eps_power": ("*a = eps * eps * nu / K;", "*a = eps * nu / K;"),
    "velocity_drop_half_Q": ("double Vx = mx + 0.5 * (Qx + p->Gx);", "double Vx = mx + 0.5 * p->Gx;"),
    "velocity_half_drag": ("double A = S + 0.5 * a;", "double A = S + a;"),
    "velocity_forchheimer_root": ("double B = 0.5 * b;", "double B = b;"),
    "pressure_uses_eps_rho": ("double r = S / eps;", "double r = S;"),
    "grad_transposed": ("sx += W[i] * EX[i] * en;", "sx += W[i] * EY[i] * en;"),
    "grad_wall_wraps": ("    if (v < 0) return 0;\n", "    if (v < 0) return v + L;\n"),
    "grad_scale": ("gx[(size_t)y * Lx + x] = sx / CS2;", "gx[(size_t)y * Lx + x] = sx;"),
    "collide_drop_pressure_source": ("double Tx = CS2 * rho * gex + Fx;", "double Tx = Fx;"),
    "collide_relax_times_tau": ("(fi - feq[i]) / p->tau", "(fi - feq[i]) * p->tau"),
    "forchheimer_u_squared": ("double Fx = p->Gx - a * ux - b * un * ux;", "double Fx = p->Gx - a * ux - b * ux * ux;"),
    "bounce_back_same_direction": ("f[OPP[i] * N + c] = fpost[i * N + c];", "f[i * N + c] = fpost[i * N + c];"),
    "stream_opposite_direction": ("f[i * N + (size_t)yt * Lx + xt] = fpost[i * N + c];",
                                  "f[OPP[i] * N + (size_t)yt * Lx + xt] = fpost[i * N + c];"),
    "weights_swapped": ("1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,", "1.0 / 9.0,  1.0 / 36.0, 1.0 / 9.0,"),
    "velocity_set_transposed": ("static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};",
                                "static const int EY[9] = {0, 0, 1, 0, -1, 1, -1, -1, 1};"),
    "init_ignores_eps": ("orc_feq(eps[c] * p->rho0,", "orc_feq(p->rho0,"),
    # open boundaries
    "inlet_velocity_sign": ("reservoir(i, eps[c0], p->rho_in, p->u_in);",
                            "reservoir(i, eps[c0], p->rho_in, -p->u_in);"),
    "reservoir_ignores_porosity": ("reservoir(i, eps[c1], p->rho_out, p->u_out);",
                                   "reservoir(i, 1.0, p->rho_out, p->u_out);"),
    # reverse-mode gradient
    "vjp_density_sign": ("*eps_bar += -rho_bar * S / (eps * eps)", "*eps_bar += rho_bar * S / (eps * eps)"),
    "vjp_half_drag": ("a_bar += 0.5 * A_bar;", "a_bar += A_bar;"),
    "vjp_forchheimer_root": ("double B_bar = den_bar * 2.0 * Vn / R;", "double B_bar = den_bar * Vn / R;"),
    "vjp_source_velocity": ("ux_bar += -cx_bar / CS2;", "ux_bar += cx_bar / CS2;"),
    "drag_derivative_sign": ("*db = -b / (1.0 - eps);", "*db = b / (1.0 - eps);"),
    "adjoint_reservoir_dropped": ("dJdeps[c0] += fbar[i * N + c0] * reservoir(i, 1.0, p->rho_in, p->u_in);",
                                  "dJdeps[c0] += 0.0;"),
    "adjoint_bounce_same_direction": ("else if (wall) pbar[i * N + c] = fbar[OPP[i] * N + c];",
                                      "else if (wall) pbar[i * N + c] = fbar[i * N + c];"),
    "adjoint_init_dropped": ("for (int i = 0; i < 9; i++) dJdeps[c] += fbar[i * N + c] * feq1[i];",
                             "for (int i = 0; i < 9; i++) dJdeps[c] += 0.0 * feq1[i];"),
    "adjoint_stencil_sign": ("dJdeps[cn] += (gxb[c] * W[i] * EX[i]", "dJdeps[cn] -= (gxb[c] * W[i] * EX[i]"),
    # sliding walls
    "wall_gain_sign": ("return 6.0 * W[j] * p->rho0 * (EX[j] * uw);",
                       "return -6.0 * W[j] * p->rho0 * (EX[j] * uw);"),
    "wall_gain_missing_factor_two": ("return 6.0 * W[j] * p->rho0 * (EX[j] * uw);",
                                     "return 3.0 * W[j] * p->rho0 * (EX[j] * uw);"),
    "wall_gain_plates_swapped": ("double uw = top ? p->uw_top : p->uw_bot;",
                                 "double uw = top ? p->uw_bot : p->uw_top;"),
    "wall_gain_ignores_porosity": ("wall_gain(p, OPP[i], yt >= Ly) * eps[c];",
                                   "wall_gain(p, OPP[i], yt >= Ly);"),
    "ywall_bounce_same_direction": ("f[OPP[i] * N + c] = fpost[i * N + c] +",
                                    "f[i * N + c] = fpost[i * N + c] +"),
    "adjoint_wall_gain_dropped": ("dJdeps[c] += fbar[OPP[i] * N + c] * wall_gain(p, OPP[i], yt >= Ly);",
                                  "dJdeps[c] += 0.0;"),
    # the objective (outlet mass flux) and the reverse pass's seed
    "objective_column_shift": [("size_t c = (size_t)y * p->Lx + (p->Lx - 1);",
                                "size_t c = (size_t)y * p->Lx + (p->Lx - 2);"),
                               ("size_t c = (size_t)y * Lx + (Lx - 1);\n        double fc[9]",
                                "size_t c = (size_t)y * Lx + (Lx - 2);\n        double fc[9]")],
    "objective_raw_momentum": ("cell_state(p, f, N, c, eps[c], gx[c], gy[c], &S, NULL, NULL, NULL, &ux, NULL, NULL,\n"
                               "                   NULL);\n        J += S * ux;",
                               "cell_state(p, f, N, c, eps[c], gx[c], gy[c], &S, &ux, NULL, NULL, NULL, NULL, NULL,\n"
                               "                   NULL);\n        J += ux;"),
    # velocity inlet / pressure outlet
    "inlet_fixed_density": ("orc_feq(ends[3 * y], p->u_in, 0.0, feq_in);",
                            "orc_feq(eps[c0] * p->rho_in, p->u_in, 0.0, feq_in);"),
    "outlet_fixed_velocity": ("orc_feq(eps[c1] * p->rho_out, ends[3 * y + 1], ends[3 * y + 2], feq_out);",
                              "orc_feq(eps[c1] * p->rho_out, p->u_in, 0.0, feq_out);"),
    "outlet_ignores_porosity": ("orc_feq(eps[c1] * p->rho_out, ends[3 * y + 1], ends[3 * y + 2], feq_out);",
                                "orc_feq(p->rho_out, ends[3 * y + 1], ends[3 * y + 2], feq_out);"),
    "outlet_drops_transverse_velocity": ("ends[3 * y + 2] = uy;", "ends[3 * y + 2] = 0.0;"),
    "outlet_velocity_from_inlet_node": [("cell_state(p, f, N, c1, eps[c1], gx[c1], gy[c1], NULL, NULL, NULL, NULL, &ux, &uy,",
                                         "cell_state(p, f, N, c0, eps[c0], gx[c0], gy[c0], NULL, NULL, NULL, NULL, &ux, &uy,")],
    "adjoint_inlet_density_dropped": ("if (EX[i] > 0) Sb[c0] += fbar[i * N + c0] * feq_in1[i];",
                                      "if (EX[i] > 0) Sb[c0] += 0.0 * feq_in1[i];"),
    "adjoint_outlet_velocity_dropped": ("uxb[c1] += fb * W[i] * S *", "uxb[c1] += 0.0 * W[i] * S *"),
    "adjoint_outlet_porosity_dropped": ("dJdeps[c1] += fb * feq_out1[i];", "dJdeps[c1] += 0.0 * feq_out1[i];"),
    "adjoint_outlet_du_sign": ("(EX[i] / CS2 + eu * EX[i] / (CS2 * CS2) - ux / CS2)",
                               "(EX[i] / CS2 + eu * EX[i] / (CS2 * CS2) + ux / CS2)"),
}


def _pairs(name):
    m = MUTANTS[name]
    return m if isinstance(m, list) else [m]


def _kill(name, tmp):
    src = open(SRC).read()
    for old, new in _pairs(name):
        assert old in src, f"mutation anchor for {name} not found"
        # the first occurrence is the forward step; the node adjoint further down
        # recomputes the same forward quantities
        src = src.replace(old, new, 1)
    path = os.path.join(tmp, name + ".c")
    with open(path, "w") as fh:
        fh.write(src)
    lib = os.path.join(tmp, name + ".so")
    subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fopenmp", "-o", lib, path, "-lm"])
    env = dict(os.environ, LBM_VANS_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_adjoint.py"),
                        os.path.join(ROOT, "tests", "test_oracle_inout.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def test_mutation_anchors_exist():
    src = open(SRC).read()
    for name in MUTANTS:
        for old, _ in _pairs(name):
            assert old in src, f"mutation anchor for {name} not found"


def test_every_mutant_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        with concurrent.futures.ThreadPoolExecutor(max_workers=6) as ex:
            results = dict(ex.map(lambda n: _kill(n, tmp), MUTANTS))
    survivors = [n for n, rc in results.items() if rc == 0]
    assert not survivors, f"mutants not caught by any pin: {survivors}"
