"""The general affine mesh (fr_mesh_elements, section 2.1: each element the
affine image of its reference element, eqs. transall / govqtrans) against
the oracle's own construction from the same vertices.  Host only: coordinates,
face pairing and the L/R rule through the C ABI; the GPU parity on these
meshes is in test_gpu_mesh_elements.py.

The test meshes are box meshes re-expressed through their element vertices
and then mapped by a global shear and rotation, with the period lattice
mapped alike: every element is affine but no Jacobian is diagonal, and the
periodic pairing runs through a sheared lattice."""

import ctypes

import numpy as np
import pytest

import paper_2401_06132_amd as frmi
from oracle.mesh import REF_VERTS, Mesh, elements_mesh

SHEAR = np.array([[np.cos(0.4), -np.sin(0.4), 0.0], [np.sin(0.4), np.cos(0.4), 0.0], [0.0, 0.0, 1.0]]) @ \
    np.array([[1.0, 0.3, 0.1], [0.0, 1.0, 0.2], [0.0, 0.0, 1.0]])


def sheared_case(dims, p, kind, A=SHEAR):
    """(vertices per type, period lattice, the box mesh it came from)."""
    mb = Mesh(*dims, p, kind)
    verts = {t: (mb.org[t][:, None, :] + np.einsum("eij,vj->evi", mb.J[t], REF_VERTS[t])) @ A.T for t in mb.types}
    return verts, mb.lattice @ A.T, mb


def _left(m):
    left = np.zeros(m.nfpts, dtype=np.int8)
    left[m.iL] = 1
    return left


@pytest.mark.parametrize("dims,p,kind", [((3, 2, 4), 2, "mixed"), ((2, 3, 2), 3, "hex"), ((2, 2, 3), 1, "prism"),
                                         ((2, 2, 3), 2, "hex_prism_pyr_tet"), ((1, 1, 1), 2, "hex")])
def test_pairing_and_left_right_match_the_oracle(dims, p, kind):
    verts, lat, mb = sheared_case(dims, p, kind)
    m = elements_mesh(p, verts, lat)
    s = frmi.Solver(None, p, "elements", verts=verts, period=lat)
    assert [b[0] for b in s.blocks()] == m.types
    for g, t in zip(s.upts_coords(), m.types):
        np.testing.assert_allclose(g, m.upts_coords(t), atol=1e-12)
    nbr, isl = s.connectivity()
    np.testing.assert_array_equal(nbr, m.partner)
    np.testing.assert_array_equal(isl, _left(m))
    # the shear moves no face to another partner: the box's own pairing (and
    # the box's L/R where its cell order numbers the elements in library
    # order -- one type, or hexahedra below prisms -- and no element pairs
    # with itself, whose L/R follows the centroids' lexicographic order)
    np.testing.assert_array_equal(m.partner, mb.partner)
    if kind in ("hex", "prism", "mixed") and min(dims) > 1:
        np.testing.assert_array_equal(_left(m), _left(mb))


def test_unsheared_vertices_reproduce_the_box_mesh():
    dims, p = (3, 2, 4), 2
    verts, lat, mb = sheared_case(dims, p, "mixed", A=np.eye(3))
    s = frmi.Solver(None, p, "elements", verts=verts, period=lat)
    b = frmi.Solver(dims, p, "mixed")
    np.testing.assert_array_equal(s.connectivity()[0], b.connectivity()[0])
    np.testing.assert_array_equal(s.connectivity()[1], b.connectivity()[1])
    for x, y in zip(s.upts_coords(), b.upts_coords()):
        np.testing.assert_allclose(x, y, atol=1e-13)


def _expect(status, verts, p=2, period=None, **phys):
    with pytest.raises(frmi.FrError, match=status):
        frmi.Solver(None, p, "elements", verts=verts, period=period, **phys)


def test_bad_meshes_are_rejected():
    verts, lat, _ = sheared_case((2, 2, 2), 2, "hex")
    # a missing element leaves faces unpaired
    _expect("FR_EINVAL", {"hex": verts["hex"][1:]}, period=lat)
    # without the period the boundary faces are unpaired
    _expect("FR_EINVAL", verts)
    # a moved vertex: no longer the affine image of the reference hexahedron
    bad = verts["hex"].copy()
    bad[0, 7] += 0.05
    _expect("FR_EINVAL", {"hex": bad}, period=lat)
    # a mirrored element has a negative Jacobian
    bad = verts["hex"].copy()
    bad[0] = bad[0][[1, 0, 3, 2, 5, 4, 7, 6]]
    _expect("FR_EINVAL", {"hex": bad}, period=lat)
    # order outside 1..4
    _expect("FR_EUNSUPPORTED", verts, p=5, period=lat)
    tv, tlat, _ = sheared_case((1, 1, 1), 2, "tet")
    _expect("FR_EUNSUPPORTED", tv, period=tlat, surface_aa=True)


def test_null_arguments_are_rejected():
    lib = frmi.load_library()
    ph = frmi.physics()
    c = ctypes.c_void_p()
    assert lib.fr_create(ctypes.byref(ph), None, ctypes.byref(c)) == 0
    try:
        counts = (ctypes.c_int64 * 4)(1, 0, 0, 0)
        ptrs = (ctypes.c_void_p * 4)(None, None, None, None)
        assert lib.fr_mesh_elements(c, 2, None, ptrs, None) == -1
        assert lib.fr_mesh_elements(c, 2, counts, None, None) == -1
        assert lib.fr_mesh_elements(c, 2, counts, ptrs, None) == -1  # a count with no vertices
        counts0 = (ctypes.c_int64 * 4)(0, 0, 0, 0)
        assert lib.fr_mesh_elements(c, 2, counts0, ptrs, None) == -1
    finally:
        lib.fr_destroy(c)
