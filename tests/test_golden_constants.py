"""The workload parameters and the oracle's time integration against the constants the
paper states (tests/golden/paper_constants.txt)."""
import math

import pytest

import synthetic as sy
from golden_data import paper_constants
from test_oracle_waves import P5

G = paper_constants()


def test_jet_workload_uses_the_papers_constants():
    p = sy.jet_params((16, 12, 8))
    assert p.prandtl == G["prandtl"]
    assert p.prandtl_sgs == G["prandtl_sgs"]
    assert p.cs == G["smagorinsky_cs"]
    assert p.k2 == G["k2"]
    assert p.k4 == G["k4"]
    assert p.mach_jet == G["jet_mach"]
    # S1 enters in reference units: S1 / T_ref with the unheated reference 288.15 K.
    assert p.suth_s1 * 288.15 == pytest.approx(G["sutherland_s1_kelvin"], rel=1e-15)


def test_jet_is_perfectly_expanded_and_unheated():
    # In the jet-exit reference units the jet has rho = 1, p = 1/gamma, T = gamma p / rho = 1.
    p = sy.jet_params((16, 12, 8))
    p_jet, rho_jet = 1.0 / p.gamma, 1.0
    t_jet = p.gamma * p_jet / rho_jet
    t_inf = p.gamma * p.p_inf / p.rho_inf
    assert p_jet / p.p_inf == pytest.approx(G["jet_pressure_ratio"], rel=1e-15)
    assert t_jet / t_inf == pytest.approx(G["jet_temperature_ratio"], rel=1e-15)


def test_runge_kutta_coefficients_and_stated_bound():
    # The wave tests pin the oracle's step to the stability polynomial P5 built from the
    # stated coefficients. Here P5 is checked against its expansion and the stated linear
    # bound: |P(iy)| <= 1 up to y = 2 sqrt(2).
    assert len(G["rk_alpha"]) == 5
    for z in (0.3, -1.2 + 0.4j, 2.5j, 2.0 + 1.0j):
        poly = 1 + z + z ** 2 / 2 + 3 * z ** 3 / 16 + z ** 4 / 32 + z ** 5 / 128
        assert abs(P5(z) - poly) < 1e-14
    bound = G["rk_cfl_bound"]
    assert bound == pytest.approx(2.0 * math.sqrt(2.0), rel=1e-15)
    for t in range(1, 201):
        y = bound * t / 200.0
        assert abs(P5(1j * y)) <= 1.0 + 1e-14
