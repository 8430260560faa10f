"""Seeded synthetic inputs: the compressible Taylor-Green vortex initial state
and the additive noise, evaluated at caller-supplied solution-point
coordinates.  This module holds no flux-reconstruction arithmetic; it is
shared by the library's benchmarks and by the tests (which feed the same
arrays to the reference oracle and to the GPU path).

Taylor-Green vortex (section 6 of the paper), with rho0 = U0 = L = 1 and
Mach 0.1 based on U0:
    v_x =  sin x cos y cos z,  v_y = -cos x sin y cos z,  v_z = 0
    p   =  p0 + (cos 2x + cos 2y)(cos 2z + 2) / 16,   p0 = 1 / (gamma Ma^2)
    rho =  p / (R T0) with R T0 = p0 / rho0  (isothermal start)
The paper prints v_y with a plus sign; the minus sign makes the field
divergence free and is the standard vortex (a reading).

Noise: an additive absolute U(-amp, amp) perturbation of every conserved
variable at every solution point, numpy PCG64(seed), drawn in the order
[element][variable][point] per element type, hex block first.
"""

import numpy as np

GAMMA = 1.4
MACH = 0.1
P0 = 1.0 / (GAMMA * MACH * MACH)
RHO0 = 1.0  # mean density of the vortex


def tgv_state(xyz, gamma=GAMMA, p0=P0):
    """Conserved TGV state at coordinates xyz (..., 3) -> (..., 5)."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    vx = np.sin(x) * np.cos(y) * np.cos(z)
    vy = -np.cos(x) * np.sin(y) * np.cos(z)
    p = p0 + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
    rho = p / p0
    E = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy)
    return np.stack([rho, rho * vx, rho * vy, np.zeros_like(x), E], axis=-1)


def element_state(coords, noise_amp=1e-3, seed=0, rng=None):
    """coords: list of per-type arrays (E_t, N_u, 3) in library/oracle order.
    Returns a list of (E_t, 5, N_u) float64 arrays (TGV + seeded noise)."""
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for c in coords:
        u = np.ascontiguousarray(tgv_state(c).transpose(0, 2, 1))
        if noise_amp:
            u += rng.uniform(-noise_amp, noise_amp, size=u.shape)
        out.append(u)
    return out


def uniform_state(shape_list, rho=1.0, v=(0.3, -0.2, 0.1), p=P0, gamma=GAMMA):
    """A constant (free-stream) state for every element of every type."""
    E = p / (gamma - 1.0) + 0.5 * rho * float(np.dot(v, v))
    vals = np.array([rho, rho * v[0], rho * v[1], rho * v[2], E])
    return [np.broadcast_to(vals[None, :, None], (E_t, 5, nu)).copy() for E_t, nu in shape_list]


def serving_requests(n=512, rate=200.0, seed=0, nmin=6, nmax=32, steps=(20, 200), orders=(2, 3, 4)):
    """The request stream of the serving workload: Poisson arrivals, mesh
    size ~ U{nmin..nmax} cubed, type ~ U{hex, prism}, order ~ U{orders},
    RK4 steps ~ U{steps}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    size = rng.integers(nmin, nmax + 1, size=n)
    etype = rng.integers(0, 2, size=n)
    order = rng.choice(np.asarray(orders), size=n)
    nsteps = rng.integers(steps[0], steps[1] + 1, size=n)
    return [dict(id=i, arrival=float(t[i]), n=int(size[i]), etype=("hex", "prism")[etype[i]],
                 p=int(order[i]), steps=int(nsteps[i]), seed=i) for i in range(n)]
