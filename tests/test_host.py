"""CPU tests of the library's host logic (no GPU): the shared library loads
and exports every symbol the header declares; the C++ reference-element
setup (bisection/Newton roots, product-formula Lagrange polynomials, PKD
triangle basis) agrees with the oracle's independent construction
(Vandermonde of Legendre products); mesh coordinates and face connectivity
agree with the oracle's coordinate-based pairing, including the L/R rule."""

import os
import re

import numpy as np
import pytest

import paper_2401_06132_amd as frmi
from oracle.elements import RefElement
from oracle.mesh import Mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    try:
        return frmi.load_library()
    except frmi.FrError as e:  # pragma: no cover
        pytest.fail(str(e))


def test_library_exports_every_declared_symbol():
    lib = _lib_or_skip()
    hdr = open(os.path.join(ROOT, "include", "fr.h")).read()
    declared = set(re.findall(r"^\s*(?:fr_status|void|const char\s*\*)\s*(fr_[a-z0-9_]+)\s*\(", hdr, re.M))
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(frmi.SYMBOLS)


@pytest.mark.parametrize("etype,name", [(0, "hex"), (1, "prism"), (2, "tet"), (3, "pyr")])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_reference_operators_match_oracle(etype, name, p):
    _lib_or_skip()
    r = RefElement(name, p)
    pairs = [("upts", r.upts), ("fpts", r.fpts), ("qpts", r.qpts), ("qwts", r.qwts), ("M0", r.M0), ("M3", r.M3),
             ("M7", r.M7), ("M8", r.M8), ("wu", r.wu), ("Dxi", r.Dg[0]), ("Deta", r.Dg[1]), ("Dzeta", r.Dg[2])]
    if name == "pyr":
        pairs += [("APd", r.Kq), ("Ku", r.Ku), ("K0", r.Ku)]
    if name == "tet":
        # no anti-aliasing: the strong form (M1 - M3 M2) as one operator per direction
        k0 = np.stack([r.Dg[d] - r.M3 @ (r.fnorm[:, d][:, None] * r.M0) for d in range(3)])
        pairs += [("K0", k0)]
    for key, ref in pairs:
        got = frmi.ref_operator(etype, p, key).reshape(ref.shape)
        scale = max(1.0, np.abs(ref).max())
        np.testing.assert_allclose(got, ref, atol=5e-14 * scale, err_msg=key)


@pytest.mark.parametrize("kind", ["hex", "prism", "mixed", "tet", "prism_tet", "hex_warp", "prism_warp", "mixed_warp",
                                  "pyr", "hex_pyr", "hex_pyr_tet", "hex_prism_pyr_tet"])
def test_mesh_coordinates_and_connectivity_match_oracle(kind):
    _lib_or_skip()
    dims = (3, 2, 4)
    s = frmi.Solver(dims, 2, kind)
    m = Mesh(*dims, 2, kind)
    got = s.upts_coords()
    assert len(got) == len(m.types)
    for g, t in zip(got, m.types):
        np.testing.assert_allclose(g, m.upts_coords(t), atol=1e-13)
    nbr, isl = s.connectivity()
    assert len(nbr) == m.nfpts
    np.testing.assert_array_equal(nbr, m.partner)
    left = np.zeros(m.nfpts, dtype=np.int8)
    left[m.iL] = 1
    np.testing.assert_array_equal(isl, left)


def test_bad_arguments_are_rejected():
    lib = _lib_or_skip()
    with pytest.raises(frmi.FrError):
        frmi.Solver(2, 5, "hex")
    with pytest.raises(frmi.FrError):
        frmi.Solver(0, 2, "hex")
    with pytest.raises(frmi.FrError):
        frmi.ref_operator(0, 2, "nope")
    assert lib.fr_create(None, None, None) != 0


def test_surface_aa_rejected_where_not_built():
    """Surface-flux anti-aliasing needs flux anti-aliasing and the fused form
    (checked before any device call)."""
    _lib_or_skip()
    with pytest.raises(frmi.FrError, match="FR_EUNSUPPORTED"):
        frmi.Solver((2, 2, 2), 3, "hex", aa=False, surface_aa=True)
    for kind in ("hex_warp", "prism_warp", "mixed_warp"):
        with pytest.raises(frmi.FrError, match="FR_EUNSUPPORTED"):
            frmi.Solver((2, 2, 2), 3, kind, aa=False)
        with pytest.raises(frmi.FrError, match="FR_EUNSUPPORTED"):
            frmi.Solver((2, 2, 2), 3, kind, form="plain")
    for kind in ("tet", "pyr", "hex_pyr"):
        with pytest.raises(frmi.FrError, match="FR_EUNSUPPORTED"):
            frmi.Solver((2, 2, 2), 3, kind, surface_aa=True)
    frmi.Solver((2, 2, 2), 3, "tet", aa=False)
    frmi.Solver((2, 2, 2), 3, "prism_tet", form="plain")
    with pytest.raises(frmi.FrError, match="FR_EUNSUPPORTED"):
        frmi.Solver((2, 2, 2), 3, "hex", form="plain", surface_aa=True)
    for kind in ("hex", "prism", "mixed"):
        frmi.Solver((2, 2, 2), 3, kind, surface_aa=True)
    with pytest.raises(frmi.FrError, match="FR_EINVAL"):
        frmi.Solver((2, 2, 2), 3, "hex_pyr_tet")


@pytest.mark.parametrize("kind", ["hex", "prism", "mixed", "tet", "prism_tet", "pyr", "hex_pyr", "hex_pyr_tet",
                                  "hex_prism_pyr_tet"])
def test_element_counts_match_oracle(kind):
    """The library's element counts per type (hexahedra, prisms, tetrahedra,
    pyramids) and its pairing match the oracle's."""
    _lib_or_skip()
    dims = (2, 3, 3) if kind.endswith("pyr_tet") else (2, 3, 2)
    s = frmi.Solver(dims, 2, kind)
    m = Mesh(*dims, 2, kind)
    counts = {"hex": s.n_hex, "prism": s.n_prism, "tet": s.n_tet, "pyr": s.n_pyr}
    for t in ("hex", "prism", "tet", "pyr"):
        assert counts[t] == m.nelem.get(t, 0)
    nbr, isl = s.connectivity()
    np.testing.assert_array_equal(nbr, m.partner)
