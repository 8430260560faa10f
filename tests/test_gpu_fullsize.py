"""GPU parity at the benchmark sizes, on sampled elements.

The full right-hand side is computed on the GPU (same library call and
launch configuration as bench.py); the oracle evaluates the RHS of a random
sample of elements (rhs_subset: the two-hop neighbourhood of each sampled
element), in extended precision.  Tolerances as in test_gpu_parity.py:
fused and plain FP64 1e-12, FP32 2e-5 (per variable, relative to the
sample's max).  Besides the benchmark configurations (hexahedra and prisms
at p = 3 and 4 in FP32, FP64 and the plain FP64 form, the mixed mesh), the tetrahedron, pyramid and four-type meshes that the
benchmark also times run here at 48^3 cells in FP32 (the matrix-core volume
kernels, with and without flux anti-aliasing).
"""

import numpy as np
import pytest

import paper_2401_06132_amd as frmi
from oracle.mesh import Mesh
from oracle.rhs import Params, rhs_subset
from paper_2401_06132_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_MESH = {}


def _mesh(kind, n, p):
    key = (kind, n, p)
    if key not in _MESH:
        _MESH.clear()
        _MESH[key] = Mesh(n, n, n, p, kind)
    return _MESH[key]


CASES = [("hex", 48, 3, "fp32"), ("hex", 48, 3, "fp64"), ("hex", 48, 3, "plain"), ("hex", 48, 4, "fp32"),
         ("hex", 48, 4, "fp64"), ("hex", 48, 4, "plain"), ("prism", 48, 3, "fp32"), ("prism", 48, 3, "fp64"),
         ("prism", 48, 4, "fp32"), ("prism", 48, 4, "fp64"), ("prism", 48, 4, "plain"),
         ("mixed", 64, 4, "fp32"), ("tet", 48, 3, "fp32"), ("tet", 48, 3, "fp32_noaa"),
         ("pyr", 48, 3, "fp32"), ("hex_prism_pyr_tet", 48, 3, "fp32")]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kind,n,p,prec", CASES)
def test_fullsize_sampled_parity(kind, n, p, prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("fullsize case", kind, n, p, prec, flush=True)
    m = _mesh(kind, n, p)
    U = inputs.element_state([m.upts_coords(t) for t in m.types], seed=0)
    form = "plain" if prec == "plain" else "fused"
    aa = not prec.endswith("_noaa")
    prec = prec.replace("_noaa", "")
    s = frmi.Solver(n, p, kind, prec="fp64" if prec == "plain" else prec, form=form, pref=inputs.P0, rho_ref=inputs.RHO0, aa=aa)
    lib_xyz = s.upts_coords()
    for t, x in zip(m.types, lib_xyz):
        np.testing.assert_allclose(x[::997], m.upts_coords(t)[::997], atol=1e-12)
    u = torch.from_numpy(np.concatenate([x.reshape(-1) for x in U])).cuda()
    du = torch.empty_like(u)
    s.rhs(u, du)
    torch.cuda.synchronize()
    got = s.split(du.cpu().numpy())
    del u, du
    rng = np.random.default_rng(12345)
    sel = {t: np.sort(rng.choice(m.nelem[t], size=96, replace=False)) for t in m.types}
    Uo = {t: x for t, x in zip(m.types, U)}
    ref = rhs_subset(m, {t: x.astype(np.longdouble) for t, x in Uo.items()}, Params(pref=inputs.P0, aa=aa), sel,
                     dtype=np.longdouble)
    tol = 2e-5 if prec == "fp32" else 1e-12
    for t, g in zip(m.types, got):
        r = ref[t]
        err = (np.abs(g[sel[t]] - r).max(axis=(0, 2)) / np.abs(r).max(axis=(0, 2))).astype(np.float64)
        print(kind, n, p, prec, t, "rel err per variable", err, flush=True)
        assert np.all(err < tol), err
