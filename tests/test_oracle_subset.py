"""The oracle's neighbourhood-restricted right-hand side (rhs_subset), which
the full-size GPU parity tests use as their reference, against the whole-mesh
rhs() on the same state.  It re-implements the kernel sequence of section 2.2
on the two-hop neighbourhood of the sampled elements, so a wrong hop count, a
neighbour lookup that misses the periodic wrap, or a mismatched L/R rule
would show here as a difference well above rounding."""

import numpy as np
import pytest

from oracle.mesh import Mesh
from oracle.rhs import Params, rhs, rhs_subset
from paper_2401_06132_amd import inputs

CASES = [
    ("hex", (3, 3, 3), 2, False, True),
    ("hex", (4, 2, 3), 3, False, True),
    ("prism", (2, 3, 2), 2, False, True),
    ("mixed", (2, 2, 4), 2, False, True),
    ("tet", (2, 2, 2), 2, False, True),
    ("pyr", (2, 2, 2), 2, False, True),
    ("hex_prism_pyr_tet", (2, 2, 3), 1, False, True),
    ("hex_warp", (3, 2, 3), 2, False, True),
    ("prism_warp", (2, 2, 2), 2, False, True),
    ("hex", (3, 3, 2), 2, True, True),
    ("mixed", (2, 2, 4), 2, True, True),
    ("hex", (3, 3, 3), 2, False, False),
    ("mixed", (2, 3, 4), 2, False, False),
]


@pytest.mark.parametrize("kind,dims,p,surf_aa,aa", CASES)
def test_rhs_subset_equals_rhs(kind, dims, p, surf_aa, aa):
    m = Mesh(*dims, p, kind, surf_aa=surf_aa)
    U = {t: u for t, u in zip(m.types, inputs.element_state([m.upts_coords(t) for t in m.types], seed=7))}
    par = Params(pref=inputs.P0, aa=aa)
    full = rhs(m, U, par)
    rng = np.random.default_rng(3)
    sel = {}
    for t in m.types:
        # the first and last elements of each type sit on the box corners,
        # so their neighbourhoods wrap the period in every direction
        pick = {0, m.nelem[t] - 1}
        pick |= set(int(e) for e in rng.choice(m.nelem[t], size=min(3, m.nelem[t]), replace=False))
        sel[t] = np.array(sorted(pick))
    sub = rhs_subset(m, U, par, sel)
    for t in m.types:
        ref = full[t][sel[t]]
        sc = np.abs(ref).max(axis=(0, 2))
        err = np.abs(sub[t] - ref).max(axis=(0, 2)) / sc
        assert np.all(err <= 1e-13), (t, err)


def test_rhs_subset_sees_its_neighbours():
    """A perturbation of one element changes the subset RHS of each of its
    face neighbours (and of itself) exactly as it changes the whole-mesh RHS.
    The element two cells away along +x is untouched: with beta = 1/2 the
    common solution of a face is the R side's state (eq. FR-conu), so the
    gradient of the element in between does not see the perturbed one."""
    m = Mesh(5, 3, 3, 2, "hex")
    U = {"hex": inputs.element_state([m.upts_coords("hex")], seed=1)[0]}
    par = Params(pref=inputs.P0)
    V = {"hex": U["hex"].copy()}
    e = 0  # corner cell: its -x neighbour is cell 4 across the period
    V["hex"][e, 1] += 1e-3 * np.linspace(0.5, 1.0, m.refs["hex"].nu)
    sel = {"hex": np.array([0, 1, 2, 4])}
    a = rhs_subset(m, U, par, sel)["hex"]
    b = rhs_subset(m, V, par, sel)["hex"]
    fa, fb = rhs(m, U, par)["hex"][sel["hex"]], rhs(m, V, par)["hex"][sel["hex"]]
    np.testing.assert_allclose(b - a, fb - fa, rtol=0, atol=1e-13 * np.abs(fa).max())
    d = np.abs(b - a).max(axis=(1, 2))
    assert d[0] > 0 and d[1] > 0 and d[3] > 0  # itself, +x and -x (wrapped) neighbours
    assert d[2] == 0.0  # two cells away
