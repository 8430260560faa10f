"""Pins for the oracle's curved (non-affine) elements: hexahedra (trilinear
maps) and prisms (triangle x line vertex maps) of a warped periodic grid.  Free-stream preservation and discrete conservation
(with the per-point det J weights), the discrete metric identity
sum_d D_d (det J J^-1)_d = 0, equality with the affine mesh when the warp is
zero, and design-order convergence to the exact time derivative of an
entropy wave."""

import numpy as np
import pytest

from oracle.mesh import Mesh
from oracle.rhs import Params, rhs
from paper_2401_06132_amd import inputs


def _integral(m, U):
    return sum(np.einsum("eu,u,evu->v", m.detJ[t], m.refs[t].wu, U[t]) for t in m.types)


@pytest.mark.parametrize("kind", ["hex_warp", "prism_warp", "mixed_warp"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_free_stream_and_conservation(kind, p):
    m = Mesh(3, 2, 3, p, kind)
    for t in m.types:
        assert np.ptp(m.detJ[t]) > 0.05 * m.detJ[t].mean()  # really non-affine
    U = {t: u for t, u in zip(m.types, inputs.uniform_state([(m.nelem[t], m.refs[t].nu) for t in m.types]))}
    for pref in (0.0, inputs.P0):
        du = rhs(m, U, Params(pref=pref))
        assert max(np.abs(du[t]).max() for t in m.types) < 1e-12 * 72 * 10
    U = {t: u for t, u in zip(m.types, inputs.element_state([m.upts_coords(t) for t in m.types]))}
    for aa in (True, False):
        du = rhs(m, U, Params(pref=inputs.P0, aa=aa))
        tot = _integral(m, du)
        scale = sum(np.einsum("eu,u,evu->v", m.detJ[t], m.refs[t].wu, np.abs(du[t])) for t in m.types)
        assert np.all(np.abs(tot) <= 1e-13 * scale)


@pytest.mark.parametrize("kind", ["hex_warp", "prism_warp"])
@pytest.mark.parametrize("p", [2, 3])
def test_metric_identity(kind, p):
    """The cofactor rows S_d = det J (J^-1)_d of the vertex maps lie in the
    solution space for p >= 2 (at most quadratic per direction), so the exact
    derivative operator gives sum_d D_d S_d = 0 to rounding."""
    m = Mesh(2, 2, 2, p, kind)
    t = m.types[0]
    r = m.refs[t]
    S = m.detJ[t][:, :, None, None] * m.Jinv[t]  # (E, N_u, 3, 3): S[e, u, d, c]
    div = sum(np.einsum("su,euc->esc", np.asarray(r.Dg[d], float), S[:, :, d, :]) for d in range(3))
    assert np.abs(div).max() < 1e-12 * np.abs(S).max()


@pytest.mark.parametrize("kind", ["hex", "prism", "mixed"])
def test_zero_warp_is_the_affine_mesh(kind):
    """Same mesh through the per-point metric path: equal to rounding (the
    1e-3 noise makes the RHS ~1e3 times smaller than the fluxes, so metric
    rounding of 1e-16 shows at ~1e-13)."""
    m0 = Mesh(3, 3, 2, 3, kind + "_warp", warp=0.0)
    ma = Mesh(3, 3, 2, 3, kind)
    U = {t: u for t, u in zip(ma.types, inputs.element_state([ma.upts_coords(t) for t in ma.types]))}
    a = rhs(m0, U, Params(pref=inputs.P0))
    b = rhs(ma, U, Params(pref=inputs.P0))
    for t in ma.types:
        assert np.abs(a[t] - b[t]).max() < 1e-12 * np.abs(b[t]).max()


def _entropy_wave(x, a=0.5, p=1.0):
    s = x[..., 0] + x[..., 1] + x[..., 2]
    rho = 1 + 0.2 * np.sin(s)
    E = p / 0.4 + 0.5 * rho * 3 * a * a
    u = np.stack([rho, rho * a, rho * a, rho * a, E], -1)
    drho = -3 * a * 0.2 * np.cos(s)
    du = np.stack([drho, a * drho, a * drho, a * drho, 1.5 * a * a * drho], -1)
    return u, du


@pytest.mark.parametrize("kind,p", [("hex_warp", 2), ("hex_warp", 3), ("prism_warp", 2), ("mixed_warp", 2)])
def test_entropy_wave_convergence(kind, p):
    errs = []
    for N in (4, 8):
        m = Mesh(N, N, N, p, kind)
        U, ex = {}, {}
        for t in m.types:
            x = m.upts_coords(t)
            U[t] = np.ascontiguousarray(np.moveaxis(_entropy_wave(x)[0], -1, 1))
            ex[t] = np.ascontiguousarray(np.moveaxis(_entropy_wave(x)[1], -1, 1))
        du = rhs(m, U, Params(mu=0.0, tau=0.0))
        errs.append(max(np.abs(du[t] - ex[t]).max() for t in m.types))
    assert np.log2(errs[0] / errs[1]) > p - 0.3
