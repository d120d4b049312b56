"""The oracle's pins must catch plausible mistakes in the oracle.

Each case below plants one mistake in a copy of the oracle's C source (a
dropped term, a wrong sign, factor or index, a transposed operand), builds
it, and runs the pin suites (tests/test_oracle_pins.py, tests/test_oracle_mrt.py
and tests/test_oracle_stencil.py, without the long runs) against that build in a
child process.  A mistake passes this test only if at least one pin fails on
it.  The unmodified source passing the same pins is the ordinary suite.
Everything runs on the CPU.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lc_oracle.c")
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_mrt.py", "tests/test_oracle_stencil.py"]

# name -> (text of the correct source, the same text with the mistake);
# each original text occurs exactly once in the source
MUTANTS = {
    # a1: Qzz dropped from the traceless completion
    "qzz_zero": ("Q[2][2] = -xx - yy;", "Q[2][2] = 0.0;"),
    # a2: first difference not halved; Laplacian centre weight 1 instead of 2
    "grad_unhalved": ("dQ[gg][a][b] = (Qp[a][b] - Qm[a][b]) / 2.0;", "dQ[gg][a][b] = (Qp[a][b] - Qm[a][b]);"),
    "lap_centre": ("L[a][b] += Qp[a][b] - 2.0 * Q0[a][b] + Qm[a][b];", "L[a][b] += Qp[a][b] - Q0[a][b] + Qm[a][b];"),
    # a3 (Eq. 4): sign of the quartic term, trace removal dropped, elastic
    # term dropped, linear coefficient
    "h_quartic_sign": ("- A0 * gam * Q[a][b] * trQ2", "+ A0 * gam * Q[a][b] * trQ2"),
    "h_no_trace": ("- A0 * gam * (trQ2 * delta / 3.0 - QQ)", "- A0 * gam * (0.0 * delta - QQ)"),
    "h_no_elastic": ("+ K * L[a][b];", ";"),
    "h_linear": ("-A0 * (1.0 - gam / 3.0) * Q[a][b]", "-A0 * (1.0 - gam / 2.0) * Q[a][b]"),
    # a4 (Eq. 6): factor of the Q:H term, sign of the antisymmetric part,
    # transposed derivative indices in the elastic term
    "tau_qh_factor": ("double t = 2.0 * xi * Qp[a][b] * QH;", "double t = xi * Qp[a][b] * QH;"),
    "tau_antisym_sign": ("t += Q[a][gg] * H[gg][b] - H[a][gg] * Q[gg][b];",
                         "t += H[a][gg] * Q[gg][b] - Q[a][gg] * H[gg][b];"),
    "tau_elastic_index": ("t -= dQ[a][gg][n] * K * dQ[b][gg][n];", "t -= dQ[gg][a][n] * K * dQ[gg][b][n];"),
    # a5: divergence taken on the first index of the stress
    "force_first_index": ("F[a] += (tau9[(a * 3 + b) * N + sp] - tau9[(a * 3 + b) * N + sm]) / 2.0;",
                          "F[a] += (tau9[(b * 3 + a) * N + sp] - tau9[(b * 3 + a) * N + sm]) / 2.0;"),
    # the same mistake in the stress entry point used by the energy balance
    "stress_force_first_index": ("F += (tau9[(a * 3 + b) * N + sp] - tau9[(a * 3 + b) * N + sm]) / 2.0;",
                                 "F += (tau9[(b * 3 + a) * N + sp] - tau9[(b * 3 + a) * N + sm]) / 2.0;"),
    # a6 (Eq. 9): velocity without the half force
    "u_no_half_force": ("u3[a * N + s] = (j[a] + F[a] / 2.0) / rho;", "u3[a * N + s] = j[a] / rho;"),
    # a7: velocity gradient differentiated along the wrong axis
    "grad_u_axis": ("size_t sp = shift(g, s, b, +1), sm = shift(g, s, b, -1);\n      G[a][b]",
                    "size_t sp = shift(g, s, a, +1), sm = shift(g, s, a, -1);\n      G[a][b]"),
    # a8 (Eqs. 1-2): vorticity transposed, Q:grad u factor, identity part of
    # Q + I/3 dropped, advection sign
    "w_transposed": ("W[a][b] = (G[a][b] - G[b][a]) / 2.0;", "W[a][b] = (G[b][a] - G[a][b]) / 2.0;"),
    "s_qgrad_factor": ("S -= 2.0 * xi * Qp[a][b] * QdU;", "S -= xi * Qp[a][b] * QdU;"),
    "s_no_identity": ("Qp[a][b] = Q[a][b] + ((a == b) ? 1.0 / 3.0 : 0.0);\n    }",
                      "Qp[a][b] = Q[a][b];\n    }"),
    "advection_sign": ("R[a][b] = Gam * H[a][b] + S - adv;", "R[a][b] = Gam * H[a][b] + S + adv;"),
    # a9-a10 (Sec. 1.2.2): half-step predictor; corrector without the average
    "predictor_half": ("qp[k] = q5[k] + R5[k]; /* step 2 */", "qp[k] = q5[k] + 0.5 * R5[k]; /* step 2 */"),
    "corrector_no_average": ("q5_out[k] = q5[k] + (R5[k] + Rp5[k]) / 2.0;", "q5_out[k] = q5[k] + Rp5[k];"),
    # a11 (Eq. 8 and the forcing term): equilibrium quadratic coefficient,
    # forcing prefactor, forcing without its velocity-dependent part
    "feq_quadratic": ("cu * cu / (2.0 * CS2 * CS2)", "cu * cu / (CS2 * CS2)"),
    "source_prefactor": ("return L->w[i] * (1.0 - 1.0 / (2.0 * tau)) * s;", "return L->w[i] * (1.0 - 1.0 / tau) * s;"),
    "source_no_cu": ("double v = L->c[i][a] / CS2 * (1.0 + cu / CS2) - u[a] / CS2;",
                     "double v = L->c[i][a] / CS2 - u[a] / CS2;"),
    # a12: streaming against the velocity
    "stream_reversed": ("site(g, x + L->c[i][0], y + L->c[i][1], z + L->c[i][2])",
                        "site(g, x - L->c[i][0], y - L->c[i][1], z - L->c[i][2])"),
    # lattice: one axis weight of D3Q19 wrong
    "d3q19_weight": ("1.0 / 3.0,  1.0 / 18.0,", "1.0 / 3.0,  1.0 / 36.0,"),
    # a13 observables: end planes of the half domain weighted 1, the half
    # domain shifted by one plane, the momentum summed with the wrong sign,
    # max |u| taken of |u|^2, S without its factor 3/2
    "observe_end_weight": ("shalf += 0.5 * S;", "shalf += S;"),
    "observe_half_start": ("long c0 = n_ax / 2, c1", "long c0 = n_ax / 2 - 1, c1"),
    "observe_mom_sign": ("mom[a] += L.c[i][a] * fi;", "mom[a] -= L.c[i][a] * fi;"),
    "observe_umax_squared": ("if (sqrt(uu) > umax) umax = sqrt(uu);", "if (uu > umax) umax = uu;"),
    "observe_s_factor": ("double S = sqrt(1.5 * qq);", "double S = sqrt(qq);"),
    # MRT: forcing relaxed with (1 - s) instead of (1 - s/2); the back-transform
    # without the 1/|m_k|^2 of the orthogonal inverse
    "mrt_forcing": ("(1.0 - op->s[k] / 2.0) * mgk", "(1.0 - op->s[k]) * mgk"),
    "mrt_inverse_norm": ("for (int k = 0; k < q; k++) ms[k] /= op->norm2[k];", ";"),
    # isotropic stencils: Laplacian without its factor 2, gradient without
    # 1/cs2, neighbours taken against the velocity, divergence on the first
    # index of the stress, velocity gradient along the wrong axis
    "iso_lap_factor": ("L[a][b] += 2.0 * iso->w[i] * (Qi[a][b] - Q0[a][b]) / CS2;",
                       "L[a][b] += iso->w[i] * (Qi[a][b] - Q0[a][b]) / CS2;"),
    "iso_grad_cs2": ("dQ[gg][a][b] += iso->w[i] * iso->c[i][gg] * Qi[a][b] / CS2;",
                     "dQ[gg][a][b] += iso->w[i] * iso->c[i][gg] * Qi[a][b];"),
    "iso_displaced_sign": ("return site(g, x + c[0], y + c[1], z + c[2]);",
                           "return site(g, x - c[0], y - c[1], z - c[2]);"),
    "iso_force_first_index": ("F[a] += iso->w[i] * iso->c[i][b] * tau9[(a * 3 + b) * N + si] / CS2;",
                              "F[a] += iso->w[i] * iso->c[i][b] * tau9[(b * 3 + a) * N + si] / CS2;"),
    "iso_grad_u_axis": ("G[a][b] += iso->w[i] * iso->c[i][b] * u3[a * N + si] / CS2;",
                        "G[a][b] += iso->w[i] * iso->c[i][a] * u3[a * N + si] / CS2;"),
}


def _run_pins(lib):
    env = dict(os.environ, LC_ORACLE_LIBRARY=lib, OMP_NUM_THREADS="2")
    cmd = [sys.executable, "-m", "pytest", *PINS, "-x", "-q", "-m", "not slow", "-p", "no:cacheprovider"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    failed = [l for l in r.stdout.splitlines() if l.startswith("FAILED")]
    return r.returncode, failed


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    src = open(SRC).read()
    d = tmp_path_factory.mktemp("mutants")
    libs = {}
    for name, (old, new) in MUTANTS.items():
        assert src.count(old) == 1, "mutation site of %s not unique or missing" % name
        c = d / (name + ".c")
        c.write_text(src.replace(old, new))
        libs[name] = oracle.compile_source(str(c), str(d / ("lib" + name + ".so")))
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        futs = {name: ex.submit(_run_pins, lib) for name, lib in libs.items()}
        return {name: f.result() for name, f in futs.items()}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(outcomes, name):
    rc, failed = outcomes[name]
    print("%s: exit %d, first failing pin: %s" % (name, rc, failed[0] if failed else "-"))
    # exit status 1: the suite ran and at least one pin failed
    assert rc == 1 and failed, "no pin failed with the mistake %r planted" % name
