"""Host observables (eqs. (Darcy), (Forchheimer), (AnalyticForce),
(frictionFactor)) on synthetic data with known answers, and the oracle's
permeability against them."""
import numpy as np

from paper_1508_02960_amd import inputs, observables as ob


def test_forchheimer_fit_recovers_known_law():
    tau = 0.8
    nu = ob.viscosity(tau)
    K, beta = 250.0, 3.5e-3
    U = np.logspace(-7, -2, 8)
    grad = nu * U / K + beta * U * U
    K_fit, b_fit, cf = ob.forchheimer_fit(grad, U, tau)
    assert abs(K_fit / K - 1) < 1e-10 and abs(b_fit / beta - 1) < 1e-8
    assert abs(cf - beta * np.sqrt(K)) < 1e-10


def test_darcy_roundtrip():
    tau, nx, D, K = 0.8, 128, 100.0, 250.0
    for re in (1e-4, 1e-2, 1.0):
        drho = ob.delta_rho_for_reynolds(re, D, tau, nx, K)
        U = K * ob.pressure_gradient(drho, nx) / ob.viscosity(tau)
        assert abs(ob.reynolds_p(U, D, tau) / re - 1) < 1e-12
        assert abs(ob.permeability(U, drho, nx, tau) / K - 1) < 1e-12


def test_drag_coefficient_and_friction_factor():
    tau, r, U = 1.0, 5.0, 1e-4
    F = 6 * np.pi * ob.viscosity(tau) * U * r * 4.0
    assert abs(ob.drag_coefficient(F, U, r, tau) - 4.0) < 1e-12
    nu = ob.viscosity(tau)
    K = 100.0
    grad = nu * U / K  # pure Darcy: F_K = 1 / Re_K
    FK, ReK = ob.friction_factor(grad, U, K, tau)
    assert abs(FK * ReK - 1) < 1e-12


def test_oracle_permeability_matches_host_formula(orc):
    shape = (10, 10, 10)
    o = orc.Oracle(shape, tau=0.9, magic=3 / 16, delta_rho=1e-5, wall="cli",
                   spheres=inputs.centred_sphere(shape, 6.0))
    o.init()
    o.step(200)
    U = o.mean_velocity()[0]
    assert abs(o.permeability() / ob.permeability(U, 1e-5, 10, 0.9) - 1) < 1e-13
