"""The single-precision split of the fused kernels, emulated on the CPU
(tests/fp32_split.py) against the oracle in extended precision.

* In float64 the kernels' split is the RHS itself rearranged (reference
  shifts, face bases and deviations, the energy flux split into an O(1) part
  and kap rho v, the mass and linear energy divergence L(rho v) in strong
  form with its interface jump term): it agrees with the oracle to
  rounding.  A wrong sign or factor anywhere in the split (kap, the
  1/2 jump term, the own-trace lift inside L) would show as an O(1e-3)
  difference.
* In float32 it meets 2e-5 per variable on 48-element samples of 12^3
  hexahedra and 10^3 prisms (p = 3, the Taylor-Green state with 1e-3
  noise), while the earlier split -- only E shifted, face values, jumps and
  all five fluxes in single precision -- misses it on density and energy:
  the noise makes the RHS ~1e3 smaller than flux magnitude times operator
  norm, and the energy flux carries gamma pref / (gamma - 1) ~ 250."""

import numpy as np
import pytest

import fp32_split
from oracle.mesh import Mesh
from oracle.rhs import Params, rhs_subset
from paper_2401_06132_amd import inputs


def _case(kind, n, p):
    m = Mesh(n, n, n, p, kind)
    U = inputs.element_state([m.upts_coords(t) for t in m.types], seed=0)[0]
    t = m.types[0]
    sel = np.sort(np.random.default_rng(5).choice(m.nelem[t], size=48, replace=False))
    par = Params(pref=inputs.P0)
    ref = rhs_subset(m, {t: U.astype(np.longdouble)}, par, {t: sel}, dtype=np.longdouble)[t].astype(np.float64)
    return m, U, par, sel, ref


def _err(du, ref):
    return np.abs(du - ref).max(axis=(0, 2)) / np.abs(ref).max(axis=(0, 2))


@pytest.mark.parametrize("kind,n", [("hex", 12), ("prism", 10)])
def test_kernel_split_is_exact_in_double(kind, n):
    m, U, par, sel, ref = _case(kind, n, 3)
    err = _err(fp32_split.rhs_split(m, U, par, sel, dtype=np.float64), ref)
    assert np.all(err < 5e-13), err


@pytest.mark.parametrize("kind,n", [("hex", 12), ("prism", 10)])
def test_kernel_split_meets_2e5_in_single(kind, n):
    m, U, par, sel, ref = _case(kind, n, 3)
    new = _err(fp32_split.rhs_split(m, U, par, sel), ref)
    old = _err(fp32_split.rhs_split(m, U, par, sel, split="energy_shift"), ref)
    print(kind, "kernels' split", new, "energy shift only", old)
    assert np.all(new < 2e-5), new
    # the earlier split misses the bar on the variables the split targets
    assert old[0] > 2e-5 and old[4] > 2e-5, old
    assert new[0] < old[0] / 20 and new[4] < old[4] / 10
