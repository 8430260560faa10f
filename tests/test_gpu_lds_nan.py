"""No kernel reads LDS that it has not written.  Before each kernel group of
the RHS (disu, volume group, interface group, enqueued one at a time with
fr_rhs_stages) the device's LDS is filled with NaN (fr_fill_lds); the result
must be finite and match the oracle to the parity tolerances of
test_gpu_parity.py.  The matrix-core products of the tetrahedron and pyramid
volume group read past a column's end where a k range is not a multiple of 4
(pyramids at p = 3: N_u = 30, tetrahedra and pyramids at p = 4); the
operator's zero padding weights those reads, which must find finite values,
whatever earlier kernels left in LDS."""

import numpy as np
import pytest

import paper_2401_06132_amd as frmi
from oracle.mesh import Mesh
from oracle.rhs import Params, rhs as oracle_rhs
from paper_2401_06132_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5}

CASES = [((2, 2, 2), p, kind) for kind in ("hex", "prism", "tet", "pyr") for p in (2, 3, 4)] + \
        [((1, 2, 3), 3, "hex_prism_pyr_tet"), ((1, 2, 3), 4, "hex_prism_pyr_tet")]


def _staged_rhs_after_nan_fills(s, flat):
    u = torch.from_numpy(flat).cuda()
    du = torch.empty_like(u)
    for mask in (1, 2, 4):
        torch.cuda.synchronize()
        frmi.fill_lds(float("nan"))
        torch.cuda.synchronize()
        s.rhs_stages(u, du, mask)
    torch.cuda.synchronize()
    return du.cpu().numpy()


@pytest.mark.parametrize("aa", [True, False])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,p,kind", CASES)
def test_rhs_after_lds_filled_with_nan(dims, p, kind, prec, aa):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("lds-nan case", dims, p, kind, prec, "aa" if aa else "noaa", flush=True)
    m = Mesh(*dims, p, kind)
    U = inputs.element_state([m.upts_coords(t) for t in m.types], seed=3)
    ref = oracle_rhs(m, {t: u.astype(np.longdouble) for t, u in zip(m.types, U)}, Params(pref=inputs.P0, aa=aa),
                     dtype=np.longdouble)
    s = frmi.Solver(dims, p, kind, prec=prec, pref=inputs.P0, rho_ref=inputs.RHO0, aa=aa)
    du = _staged_rhs_after_nan_fills(s, np.concatenate([x.reshape(-1) for x in U]))
    assert np.all(np.isfinite(du)), "non-finite output"
    err = np.max([(np.abs(g - ref[t]).max(axis=(0, 2)) / np.abs(ref[t]).max(axis=(0, 2))).astype(np.float64)
                  for g, t in zip(s.split(du), m.types)], axis=0)
    print("rel err per variable", err, flush=True)
    assert np.all(err < TOL[prec]), err


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,p,kind,saa", [((2, 2, 2), 3, "hex", True), ((2, 2, 2), 4, "hex", True),
                                              ((2, 2, 2), 3, "prism", True), ((2, 2, 2), 4, "prism", True),
                                              ((2, 2, 2), 3, "hex_warp", False), ((2, 2, 2), 4, "hex_warp", False),
                                              ((2, 2, 2), 3, "prism_warp", False)])
def test_surface_aa_and_curved_after_lds_filled_with_nan(dims, p, kind, saa, prec):
    """The same for the surface-flux anti-aliasing and curved-element kernels
    (curved FP32 held to 1e-4, as in test_gpu_parity.py)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("lds-nan case", dims, p, kind, prec, "saa" if saa else "", flush=True)
    m = Mesh(*dims, p, kind, surf_aa=saa)
    U = inputs.element_state([m.upts_coords(t) for t in m.types], seed=4)
    ref = oracle_rhs(m, {t: u.astype(np.longdouble) for t, u in zip(m.types, U)}, Params(pref=inputs.P0),
                     dtype=np.longdouble)
    s = frmi.Solver(dims, p, kind, prec=prec, pref=inputs.P0, rho_ref=inputs.RHO0, surface_aa=saa)
    du = _staged_rhs_after_nan_fills(s, np.concatenate([x.reshape(-1) for x in U]))
    assert np.all(np.isfinite(du)), "non-finite output"
    err = np.max([(np.abs(g - ref[t]).max(axis=(0, 2)) / np.abs(ref[t]).max(axis=(0, 2))).astype(np.float64)
                  for g, t in zip(s.split(du), m.types)], axis=0)
    tol = 1e-4 if (prec == "fp32" and "warp" in kind) else TOL[prec]
    print("rel err per variable", err, flush=True)
    assert np.all(err < tol), err
