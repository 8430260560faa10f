"""GPU parity on general affine meshes (fr_mesh_elements): box meshes
re-expressed through their vertices and mapped by a global shear and
rotation (test_mesh_elements.sheared_case).  No Jacobian is diagonal, so the
hexahedral kernels take their general-metric form (J^-T on the gradient and
det J J^-1 on the flux) and the prism, tetrahedron and pyramid kernels see
rotated normals.  The state is the Taylor-Green vortex of the unmapped box
at each solution point, so it is periodic on the mapped lattice.
Tolerances as in test_gpu_parity.py: FP64 1e-12, FP32 2e-5."""

import numpy as np
import pytest

import paper_2401_06132_amd as frmi
from oracle.mesh import elements_mesh
from oracle.rhs import Params, rhs as oracle_rhs, rk4_step as oracle_rk4
from paper_2401_06132_amd import inputs
from test_mesh_elements import sheared_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5}


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _setup(dims, p, kind, surf_aa=False):
    verts, lat, mb = sheared_case(dims, p, kind)
    m = elements_mesh(p, verts, lat, surf_aa=surf_aa)
    U = inputs.element_state([mb.upts_coords(t) for t in mb.types], seed=2)
    return verts, lat, m, U


def _rel_err(got, ref):
    return np.max([(np.abs(g - r).max(axis=(0, 2)) / np.abs(r).max(axis=(0, 2))).astype(np.float64)
                   for g, r in zip(got, ref)], axis=0)


CASES = [((3, 2, 4), 3, "mixed"), ((2, 3, 3), 4, "hex"), ((3, 3, 2), 2, "hex"), ((2, 2, 3), 3, "prism"),
         ((2, 2, 3), 2, "hex_prism_pyr_tet"), ((1, 2, 3), 3, "hex_prism_pyr_tet")]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("aa,saa", [(True, False), (False, False), (True, True)])
@pytest.mark.parametrize("dims,p,kind", CASES)
def test_rhs_parity_general_affine_mesh(dims, p, kind, aa, saa, prec):
    _need_gpu()
    if saa and "tet" in kind:
        pytest.skip("surface-flux anti-aliasing is not built for tetrahedra and pyramids")
    print("elements case", dims, p, kind, "aa" if aa else "noaa", "saa" if saa else "", prec, flush=True)
    verts, lat, m, U = _setup(dims, p, kind, surf_aa=saa)
    par = Params(pref=inputs.P0, aa=aa)
    ref = oracle_rhs(m, {t: u.astype(np.longdouble) for t, u in zip(m.types, U)}, par, dtype=np.longdouble)
    s = frmi.Solver(None, p, "elements", verts=verts, period=lat, prec=prec, pref=inputs.P0, rho_ref=inputs.RHO0,
                    aa=aa, surface_aa=saa)
    u = torch.from_numpy(np.concatenate([x.reshape(-1) for x in U])).cuda()
    du = torch.empty_like(u)
    s.rhs(u, du)
    torch.cuda.synchronize()
    err = _rel_err(s.split(du.cpu().numpy()), [ref[t] for t in m.types])
    print("rel err per variable", err, flush=True)
    assert np.all(err < TOL[prec]), err


def test_general_mesh_free_stream_conservation_and_rk4():
    _need_gpu()
    dims, p, kind = (3, 2, 4), 3, "mixed"
    verts, lat, m, U = _setup(dims, p, kind)
    s = frmi.Solver(None, p, "elements", verts=verts, period=lat, pref=inputs.P0, rho_ref=inputs.RHO0)
    U0 = inputs.uniform_state([(E, nu) for _, E, nu in s.blocks()])
    u = torch.from_numpy(np.concatenate([x.reshape(-1) for x in U0])).cuda()
    du = torch.empty_like(u)
    s.rhs(u, du)
    assert du.abs().max().item() < 1e-12 * 72 * 10
    Uo = {t: x for t, x in zip(m.types, U)}
    for _ in range(3):
        Uo = oracle_rk4(m, Uo, Params(pref=inputs.P0), 1e-3)
    s.set_state(np.concatenate([x.reshape(-1) for x in U]))
    c0 = s.integrals()
    s.rk4(1e-3, 3)
    for got, t, x in zip(s.split(s.get_state()), m.types, U):
        d_ref = Uo[t] - x
        err = np.abs((got - x) - d_ref).max(axis=(0, 2)) / np.abs(d_ref).max(axis=(0, 2))
        print("general mesh rk4 rel err of the state change", t, err)
        assert np.all(err < 1e-11)
    c1 = s.integrals()
    assert np.all(np.abs(c1 - c0) <= 1e-12 * np.abs(c0).max())
