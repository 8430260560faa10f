"""Pins for the oracle's point-wise physics: closed-form fluxes of simple
fields, consistency and antisymmetry of the interface fluxes, and the
equivalence of the reference-state and textbook forms."""

import numpy as np
import pytest

from oracle import physics


def _state(rng, n=7):
    rho = 1.0 + 0.2 * rng.random(n)
    v = rng.standard_normal((3, n))
    p = 50.0 + 10 * rng.random(n)
    E = p / 0.4 + 0.5 * rho * np.sum(v * v, axis=0)
    return np.concatenate([rho[None], rho[None] * v, E[None]]), rho, v, p


def test_inviscid_flux_closed_form():
    rng = np.random.default_rng(0)
    u, rho, v, p = _state(rng)
    gas = physics.Gas(pref=0.0)
    f = physics.inviscid_flux(u, gas)
    E = u[4]
    for d in range(3):
        np.testing.assert_allclose(f[d, 0], rho * v[d], rtol=1e-14)
        for i in range(3):
            np.testing.assert_allclose(f[d, 1 + i], rho * v[d] * v[i] + (p if i == d else 0), rtol=1e-13)
        np.testing.assert_allclose(f[d, 4], v[d] * (E + p), rtol=1e-13)


def test_reference_state_form_equals_textbook():
    rng = np.random.default_rng(1)
    u, rho, v, p = _state(rng)
    g0 = physics.Gas(pref=0.0)
    g1 = physics.Gas(pref=45.0)
    up = u.copy()
    up[4] -= g1.eref
    f0, f1 = physics.inviscid_flux(u, g0), physics.inviscid_flux(up, g1)
    for d in range(3):
        f1[d, 1 + d] += 45.0
    np.testing.assert_allclose(f1, f0, rtol=1e-13)
    q = rng.standard_normal((3, 5, u.shape[1]))
    np.testing.assert_allclose(physics.viscous_flux(up, q, g1), physics.viscous_flux(u, q, g0), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(physics.sound_speed(up, g1), np.sqrt(1.4 * p / rho), rtol=1e-13)


def test_viscous_flux_of_linear_velocity_and_temperature_fields():
    """Uniform density, v = A x (constant velocity gradient) and a pressure
    gradient: stress and heat flux have closed forms."""
    rng = np.random.default_rng(2)
    A = rng.standard_normal((3, 3))  # d v_i / d x_j = A[i, j]
    gp = rng.standard_normal(3)
    x = rng.standard_normal((3, 5))
    rho, p = 1.3, 40.0
    v = A @ x
    E = p / 0.4 + 0.5 * rho * np.sum(v * v, axis=0)
    u = np.concatenate([np.full((1, 5), rho), rho * v, E[None]])
    q = np.zeros((3, 5, 5))
    for j in range(3):
        q[j, 1:4] = rho * A[:, j][:, None]  # d(rho v_i)/dx_j
        # dE/dx_j = dp/dx_j / (gamma-1) + rho v . dv/dx_j
        q[j, 4] = gp[j] / 0.4 + rho * np.sum(v * A[:, j][:, None], axis=0)
    gas = physics.Gas(mu=0.3, prandtl=0.71, pref=0.0)
    f = physics.viscous_flux(u, q, gas)
    div = np.trace(A)
    for d in range(3):
        assert np.allclose(f[d, 0], 0.0)
        for i in range(3):
            T = 0.3 * (A[i, d] + A[d, i]) - (2 / 3) * 0.3 * div * (i == d)
            np.testing.assert_allclose(f[d, 1 + i], T, rtol=1e-12, atol=1e-14)
        T_row = np.array([0.3 * (A[i, d] + A[d, i]) - (2 / 3) * 0.3 * div * (i == d) for i in range(3)])
        # c_p grad T = gamma/(gamma-1) grad(p/rho); rho uniform
        heat = 0.3 / 0.71 * 1.4 / 0.4 * gp[d] / rho
        np.testing.assert_allclose(f[d, 4], np.sum(v * T_row[:, None], axis=0) + heat, rtol=1e-12)


@pytest.mark.parametrize("beta", [0.5, 0.0, -0.5, 0.2])
def test_common_flux_consistency_and_antisymmetry(beta):
    rng = np.random.default_rng(3)
    gas = physics.Gas(mu=0.01, pref=0.0)
    uL, _, _, _ = _state(rng)
    uR, _, _, _ = _state(rng)
    qL, qR = rng.standard_normal((2, 3, 5, uL.shape[1]))
    n = rng.standard_normal((3, uL.shape[1]))
    n /= np.linalg.norm(n, axis=0)
    # consistency: identical states give the physical normal flux
    F = physics.common_normal_flux(uL, uL, qL, qL, n, gas, beta, 0.1)
    fe, fv = physics.inviscid_flux(uL, gas), physics.viscous_flux(uL, qL, gas)
    np.testing.assert_allclose(F, np.einsum("dvp,dp->vp", fe - fv, n), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(physics.common_solution(uL, uL, beta), uL, rtol=1e-15)
    # swapping the sides (and the normal, and beta) negates the flux
    F1 = physics.common_normal_flux(uL, uR, qL, qR, n, gas, beta, 0.1)
    F2 = physics.common_normal_flux(uR, uL, qR, qL, -n, gas, -beta, 0.1)
    np.testing.assert_allclose(F1, -F2, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(physics.common_solution(uL, uR, beta), physics.common_solution(uR, uL, -beta),
                               rtol=1e-15)


def test_rusanov_and_penalty_are_dissipative():
    """For a pure density jump at rest, the normal mass flux must point from
    the denser side to the lighter side (Rusanov and penalty both add
    +(uL - uR) terms)."""
    gas = physics.Gas(mu=0.0, pref=0.0)
    p = 1.0
    uL = np.array([[1.2], [0], [0], [0], [p / 0.4]])
    uR = np.array([[1.0], [0], [0], [0], [p / 0.4]])
    q = np.zeros((3, 5, 1))
    n = np.array([[1.0], [0], [0]])
    F = physics.common_normal_flux(uL, uR, q, q, n, gas, 0.5, 0.1)
    s = max(np.sqrt(1.4 / 1.2), np.sqrt(1.4 / 1.0))
    np.testing.assert_allclose(F[0, 0], 0.5 * s * 0.2 + 0.1 * 0.2, rtol=1e-14)
