"""The numbers the paper prints (tests/golden/paper_values.json) against the
closed forms of its own model, on the CPU.

- The parameter set the package calls the paper's is the printed one.
- At the printed coexistence temperature the uniaxial bulk free energy of
  Eq. (3), minimised here independently of the oracle and the library, has
  its nematic minimum at the printed S_n = 1/3 and at the isotropic free
  energy (coexistence), and the correlation length of Eq. (10) is the
  printed lambda = 2.
- The printed bulk limits lie beyond the mean-field spinodals of Eq. (3):
  no nematic minimum below 8/3 (so all isotropic below 2.65) and an unstable
  isotropic state above 3 (so all nematic above 3.1).
- The printed static temperature of the R = 25 circle agrees with the
  balance of curvature-driven shrinking (Allen-Cahn, speed Gamma K / R for
  the one-constant elasticity) against the flat front's travelling-wave
  speed (10/9) Gamma A0 lambda (gamma - 2.7) to within 10%.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1907_13415_amd import inputs

with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.json")) as _fh:
    PRINTED = json.load(_fh)
P = PRINTED["parameters"]
FLAT = PRINTED["flat_interface"]
CIRCLE = PRINTED["circular_interface"]


def bulk_free_energy(S, gamma, A0):
    """Eq. (3) without gradients for Q = S (n n - I/3): tr Q^2 = 2 S^2 / 3,
    tr Q^3 = 2 S^3 / 9."""
    tr2, tr3 = 2.0 * S * S / 3.0, 2.0 * S ** 3 / 9.0
    return A0 / 2.0 * (1.0 - gamma / 3.0) * tr2 - A0 * gamma / 3.0 * tr3 + A0 * gamma / 4.0 * tr2 * tr2


def nematic_minimum(gamma, A0):
    """Largest local minimum S > 0 of the bulk free energy, or None."""
    # dF/dS as a polynomial in S, from the coefficients of F
    F = np.polynomial.Polynomial([0.0, 0.0, A0 / 3.0 * (1.0 - gamma / 3.0), -2.0 * A0 * gamma / 27.0,
                                  A0 * gamma / 9.0])
    d1, d2 = F.deriv(1), F.deriv(2)
    mins = [r.real for r in d1.roots() if abs(r.imag) < 1e-12 and r.real > 1e-9 and d2(r.real) > 0]
    return max(mins) if mins else None


def test_paper_parameter_set_is_the_printed_one():
    A0, gamma, K, Gamma, xi, tau = inputs.PAPER_PARAMS
    assert (A0, K, Gamma, xi, tau) == (P["A0"], P["K"], P["Gamma"], P["xi"], P["tau"])
    assert gamma == FLAT["gamma_coexistence"]


def test_coexistence_order_parameter_and_correlation_length():
    g, A0, K = FLAT["gamma_coexistence"], P["A0"], P["K"]
    Sn = nematic_minimum(g, A0)
    assert Sn is not None and abs(Sn - FLAT["S_n_at_coexistence"]) < 1e-12
    # coexistence: the nematic minimum has the free energy of the isotropic one
    assert abs(bulk_free_energy(Sn, g, A0)) < 1e-15
    # and it is coexistence only there: above it the nematic state is lower
    assert bulk_free_energy(nematic_minimum(g + 1e-3, A0), g + 1e-3, A0) < 0.0
    assert bulk_free_energy(nematic_minimum(g - 1e-3, A0), g - 1e-3, A0) > 0.0
    lam = math.sqrt(27.0 * K / (A0 * g))
    assert abs(lam - FLAT["lambda_at_coexistence"]) < 1e-12


@pytest.mark.parametrize("gamma", [2.0, 2.6, 2.65])
def test_no_nematic_state_at_or_below_the_isotropic_limit(gamma):
    assert gamma <= FLAT["gamma_all_isotropic_below"]
    assert nematic_minimum(gamma, P["A0"]) is None
    assert gamma < 8.0 / 3.0


@pytest.mark.parametrize("gamma", [3.1, 3.3])
def test_isotropic_state_unstable_at_or_above_the_nematic_limit(gamma):
    assert gamma >= FLAT["gamma_all_nematic_above"]
    # curvature of F at S = 0 is A0 (1 - gamma/3) * 2/3
    h = 1e-4
    curv = (bulk_free_energy(h, gamma, P["A0"]) - 2 * bulk_free_energy(0.0, gamma, P["A0"])
            + bulk_free_energy(-h, gamma, P["A0"])) / h ** 2
    assert curv < 0.0 and gamma > 3.0


def test_static_circle_temperature_balances_curvature():
    A0, K, Gamma = P["A0"], P["K"], P["Gamma"]
    lam = FLAT["lambda_at_coexistence"]
    R = CIRCLE["radius"]
    shrink = Gamma * K / R
    per_dgamma = 10.0 / 9.0 * Gamma * A0 * lam
    dg_est = shrink / per_dgamma
    dg_printed = CIRCLE["gamma_near_static"] - FLAT["gamma_coexistence"]
    assert dg_printed > 0.0  # a nematic nucleus needs a supercooled melt to stay
    assert abs(dg_est / dg_printed - 1.0) < 0.10, (dg_est, dg_printed)
