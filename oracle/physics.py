"""Point-wise physics of the compressible Navier-Stokes equations.
Test infrastructure only.

Conventions: a state array u has the conserved variables on axis 0,
u = [rho, rho v_x, rho v_y, rho v_z, E]  (eq. ucons); a gradient array q has
the physical direction on axis 0 and the variable on axis 1.  Fluxes have
the physical direction on axis 0 and the variable on axis 1.

Reference-state form.  With a constant reference pressure p_ref, the energy
stored and operated on is E' = E - p_ref/(gamma-1); the momentum flux uses
p' = p - p_ref (the constant p_ref * I flux has zero discrete divergence:
its volume and interface contributions cancel for affine elements) and the
energy flux is v (E' + p' + gamma p_ref/(gamma-1)) = v (E + p).  p_ref = 0 is
the textbook form of eqs. fluxe / fluxv.  The two forms are the same
function; the tests check that they agree to rounding.
"""

import numpy as np


class Gas:
    def __init__(self, gamma=1.4, prandtl=0.71, mu=6.25e-4, pref=0.0):
        self.gamma, self.prandtl, self.mu, self.pref = gamma, prandtl, mu, pref

    @property
    def eref(self):
        return self.pref / (self.gamma - 1.0)

    @property
    def href(self):
        return self.gamma * self.pref / (self.gamma - 1.0)


def primitives(u, gas):
    """rho, velocity (3, ...), perturbation pressure p' = p - p_ref."""
    rho = u[0]
    v = u[1:4] / rho
    pp = (gas.gamma - 1.0) * (u[4] - 0.5 * np.sum(u[1:4] * v, axis=0))
    return rho, v, pp


def inviscid_flux(u, gas):
    """f^e of eq. fluxe in reference-state form; shape (3, 5, ...)."""
    rho, v, pp = primitives(u, gas)
    f = np.empty((3,) + u.shape, dtype=u.dtype)
    h = u[4] + pp + gas.href
    for d in range(3):
        f[d, 0] = u[1 + d]
        for i in range(3):
            f[d, 1 + i] = u[1 + d] * v[i]
        f[d, 1 + d] += pp
        f[d, 4] = v[d] * h
    return f


def viscous_flux(u, q, gas):
    """f^v of eq. fluxv: stress T = mu (grad v + grad v^T) - 2/3 mu div v I,
    heat flux phi = mu c_p / Pr grad T.  The printed temperature relation has
    the wrong sign (1/(1-gamma)); the perfect-gas reading T = p/((gamma-1) c_v rho)
    gives c_p grad T = gamma grad e with e = E/rho - |v|^2/2.  Shape (3, 5, ...)."""
    g, mu = gas.gamma, gas.mu
    rho, v, _ = primitives(u, gas)
    grho = q[:, 0]
    gm = q[:, 1:4]  # gm[d, i] = d_d (rho v_i)
    gv = (gm - v[None, :] * grho[:, None]) / rho  # gv[d, i] = d_d v_i
    div = gv[0, 0] + gv[1, 1] + gv[2, 2]
    etot = u[4] + gas.eref
    ge = (q[:, 4] - (etot / rho) * grho) / rho - np.sum(v[None, :] * gv, axis=1)
    f = np.zeros((3,) + u.shape, dtype=u.dtype)
    for d in range(3):
        for i in range(3):
            t = mu * (gv[d, i] + gv[i, d])
            if i == d:
                t = t - (2.0 / 3.0) * mu * div
            f[d, 1 + i] = t
        f[d, 4] = sum(v[i] * f[d, 1 + i] for i in range(3)) + mu * g / gas.prandtl * ge[d]
    return f


def sound_speed(u, gas):
    rho, v, pp = primitives(u, gas)
    return np.sqrt(gas.gamma * (pp + gas.pref) / rho)


def common_solution(uL, uR, beta):
    """LDG common solution C(uL, uR) = (1/2 - beta) uL + (1/2 + beta) uR (eq. FR-conu)."""
    return (0.5 - beta) * uL + (0.5 + beta) * uR


def common_normal_flux(uL, uR, qL, qR, nL, gas, beta, tau):
    """Common normal flux w.r.t. the unit normal nL (eq. FR-comm_flux).

    Inviscid: Rusanov, 1/2 (f^e_L + f^e_R).n + 1/2 s (uL - uR) with
    s = max(|vL.n| + cL, |vR.n| + cR) (the paper names Rusanov's solver but not
    its wave-speed estimate; this is the reading).
    Viscous: LDG, n.((1/2+beta) f^v_L + (1/2-beta) f^v_R), with the penalty
    tau (uL - uR) taken with the same sign as the Rusanov dissipation (the
    printed placement inside F^v, which enters with a minus sign, would make
    it anti-dissipative; this is the reading).
    Total: F = F^e - F^v_LDG + tau (uL - uR).  Arrays: u (5, P), q (3, 5, P),
    nL (3, P)."""
    feL = inviscid_flux(uL, gas)
    feR = inviscid_flux(uR, gas)
    fvL = viscous_flux(uL, qL, gas)
    fvR = viscous_flux(uR, qR, gas)
    _, vL, _ = primitives(uL, gas)
    _, vR, _ = primitives(uR, gas)
    vnL = np.sum(vL * nL, axis=0)
    vnR = np.sum(vR * nL, axis=0)
    s = np.maximum(np.abs(vnL) + sound_speed(uL, gas), np.abs(vnR) + sound_speed(uR, gas))
    fe = 0.5 * np.einsum("dvp,dp->vp", feL + feR, nL) + 0.5 * s * (uL - uR)
    fv = np.einsum("dvp,dp->vp", (0.5 + beta) * fvL + (0.5 - beta) * fvR, nL)
    return fe - fv + tau * (uL - uR)
