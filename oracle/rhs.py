"""Semi-discrete right-hand side du/dt = R(u) and RK4.  Test infrastructure only.

Follows the paper's kernel formulation (section 2.2, kernel order of PyFR
v1.11.0), with dense operators and no fusion:
   1 disu          U^f  = M0 U
   2 con_u         C    = (1/2 - beta) uL + (1/2 + beta) uR, written to both sides
   3,4 tgradpcoru/tgradcoru   Q~ = M4 U + M6 (C - U^f)
        (eq. Qsubs; its last line carries a sign slip, the first line is used)
   5 gradcoru      Q    = J^-T Q~
   6 gradcoru_fpts Q^f  = M5 Q = (I3 x M0) Q
   7,8 gradcoru_qpts/uqpts   Q^q = M10 Q,  U^q = M7 U
   9 tdisf         F~^q = det J  J^-1 f(U^q, Q^q)
  10 tdivtpcorf    R~   = (M1 - M3 M2) M9 F~^q, applied literally:
                   F~^u = M8 F~^q (per component), then
                   R~ = sum_d D_d F~^u_d - M3 (sum_d nhat_d M0 F~^u_d)
                   Pyramids: the pyramid space (rational, see basis.py) is
                   not closed under differentiation, so this strong form is
                   not conservative there and differs from the weak form it
                   equals for the other element types.  Pyramids take the
                   weak form, R~ = sum_d -Mass^-1 Dq_d^T W_q F~^q_d (the
                   DG-equivalent reading of FR with DG correction
                   functions); without anti-aliasing F~^q = M7 F~^u.
  11 comm_flux     D~ = mag_L F(uL, uR, qL, qR, nL) on L, -mag_R F on R
                   (mag: each side's own area factor |det J J^-T nhat|)
  12 tdivtconf     R~  += M3 D~
  13 negdivconf    R   = -R~ / det J
Affine elements: J, det J and J^-1 are constant per element.  Curved
elements (trilinear maps): J^-T at the solution points (step 5), det J J^-1
at the quadrature points (step 9; at the solution points without AA), det J
at the solution points (step 13), and the normals and area factors of every
flux point from J there.

Without flux anti-aliasing (the paper's "AA off" configuration) steps 7, 8
and the projection M8 are absent: tdisf evaluates the flux at the solution
points from U and Q, and that F~^u enters step 10 directly.

Surface-flux anti-aliasing needs no change here: it is a property of the
mesh's reference elements (flux points at the face quadrature points, with
M0, M3 and M6 rebuilt), and every step above applies unchanged.

Arrays: the state of element type t is U[t] with shape (E_t, 5, N_u)
(element, variable, solution point).
"""

import numpy as np

from . import physics


class Params:
    """Physics and scheme parameters.  Defaults are the Taylor-Green setup:
    gamma 1.4, Pr 0.71, Re 1600 (mu = 1/1600 with rho0 = U0 = L = 1), LDG
    beta = 1/2, tau = 0.1, reference pressure 0 (textbook form)."""

    def __init__(self, gamma=1.4, prandtl=0.71, mu=1.0 / 1600.0, beta=0.5, tau=0.1, pref=0.0, aa=True):
        self.gas = physics.Gas(gamma, prandtl, mu, pref)
        self.beta, self.tau = beta, tau
        self.aa = aa  # flux anti-aliasing on (default) or off


def _flat(arrs, mesh, tail):
    return np.concatenate([arrs[t].reshape((-1,) + tail) for t in mesh.types])


def _unflat(flat, mesh, t, tail):
    r = mesh.refs[t]
    o = mesh.foff[t]
    return flat[o:o + mesh.nelem[t] * r.nf].reshape((mesh.nelem[t], r.nf) + tail)


def _divergence(r, u, q, detj, jinv, gas, aa, cast):
    """Steps 7-10: the volume part of R~, (E, N_u, 5)."""
    if r.etype == "pyr":
        f = _volume_flux(r, u, q, detj, jinv, gas, aa, cast, project=False)
        return np.einsum("dsq,edqv->esv", cast(r.Kq if aa else r.Ku), f)
    fu = _volume_flux(r, u, q, detj, jinv, gas, aa, cast)
    div = np.einsum("dsu,eduv->esv", cast(r.Dg), fu)  # M1
    nf = np.einsum("fd,fu,eduv->efv", cast(r.fnorm), cast(r.M0), fu)  # M2
    return div - np.einsum("uf,efv->euv", cast(r.M3), nf)  # - M3 M2


def _volume_flux(r, u, q, detj, jinv, gas, aa, cast, project=True):
    """Transformed flux F~ at the solution points, (E, 3, N_u, 5).
    u: (E, N_u, 5) state (reference form), q: (E, 3, N_u, 5) gradients.
    With flux anti-aliasing: U^q = M7 U, Q^q = M10 Q (steps 7, 8), the flux
    at the quadrature points (step 9) and its projection M9 = I3 x M8 (first
    factor of step 10).  Without: the flux at the solution points.
    detj, jinv: per element ((E,), (E, 3, 3)) on affine meshes, or at the
    points where the flux is evaluated ((E, N), (E, N, 3, 3)) on curved ones."""
    if aa:
        uq = np.einsum("qu,euv->vqe", cast(r.M7), u)  # 8 uqpts
        qq = np.einsum("qs,ecsv->cvqe", cast(r.M7), q)  # 7 gradcoru_qpts
    else:
        uq = np.ascontiguousarray(u.transpose(2, 1, 0))  # (5, N_u, E)
        qq = np.ascontiguousarray(q.transpose(1, 3, 2, 0))  # (3, 5, N_u, E)
    f = physics.inviscid_flux(uq, gas) - physics.viscous_flux(uq, qq, gas)  # 9 tdisf
    if np.ndim(detj) == 2:
        ft = np.einsum("eq,eqdc,cvqe->edqv", cast(detj), cast(jinv), f)
    else:
        ft = np.einsum("e,edc,cvqe->edqv", cast(detj), cast(jinv), f)
    if aa and project:
        return np.einsum("uq,edqv->eduv", cast(r.M8), ft)  # 10 tdivtpcorf: M9 (I3 x M8)
    return ft


def _sel(a, sel):
    return a if sel is None else a[sel]


def _to_physical(mesh, t, qt, sel, cast):
    """q = J^-T q~ at the solution points (eq. FR-gradcoru); qt (E, 3, N_u, 5)."""
    if mesh.curved:
        return np.einsum("esdc,edsv->ecsv", cast(_sel(mesh.Jinv[t], sel)), qt)
    return np.einsum("edc,edsv->ecsv", cast(_sel(mesh.Jinv[t], sel)), qt)


def _flux_metrics(mesh, t, aa, sel):
    """det J and J^-1 where the flux is evaluated: per element on affine
    meshes; at the quadrature points (AA) or solution points on curved ones."""
    if mesh.curved and aa:
        return _sel(mesh.detJq[t], sel), _sel(mesh.Jinvq[t], sel)
    return _sel(mesh.detJ[t], sel), _sel(mesh.Jinv[t], sel)


def _detj_u(mesh, t, sel, cast):
    """det J broadcast against (E, N_u, 5): per element, or per solution point."""
    d = cast(_sel(mesh.detJ[t], sel))
    return d[:, :, None] if mesh.curved else d[:, None, None]


def rhs(mesh, U, par, dtype=None):
    """Return du = R(u) for every element type (dict of (E_t, 5, N_u) arrays)."""
    gas, beta, tau = par.gas, par.beta, par.tau
    if dtype is None:
        dtype = U[mesh.types[0]].dtype
    cast = lambda a: np.asarray(a, dtype=dtype)  # noqa: E731
    Up, Uf = {}, {}
    for t in mesh.types:
        u = cast(U[t]).transpose(0, 2, 1).copy()  # (E, Nu, 5)
        u[:, :, 4] -= cast(gas.eref)  # reference-state form (E' = E - E_ref)
        Up[t] = u
        Uf[t] = np.einsum("fu,euv->efv", cast(mesh.refs[t].M0), u)  # 1 disu
    ufa = _flat(Uf, mesh, (5,))
    uL, uR = ufa[mesh.iL], ufa[mesh.iR]
    ca = np.empty_like(ufa)
    c = physics.common_solution(uL, uR, beta)  # 2 con_u
    ca[mesh.iL] = c
    ca[mesh.iR] = c
    Q, Qf, Rt = {}, {}, {}
    for t in mesh.types:
        r = mesh.refs[t]
        C = _unflat(ca, mesh, t, (5,))
        qt = np.einsum("dsu,euv->edsv", cast(r.Dg), Up[t])  # 3 tgradpcoru (M4 part)
        qt += np.einsum("dsf,efv->edsv", cast(r.M6), C - Uf[t])  # 4 tgradcoru
        q = _to_physical(mesh, t, qt, None, cast)  # 5 gradcoru (J^-T)
        Q[t] = q
        Qf[t] = np.einsum("fs,ecsv->efcv", cast(r.M0), q)  # 6 gradcoru_fpts
    for t in mesh.types:
        r = mesh.refs[t]
        E = mesh.nelem[t]
        rt = np.empty((E, r.nu, 5), dtype=dtype)
        chunk = max(1, int(2.0e7 // (r.nq * 20)))
        for e0 in range(0, E, chunk):
            sl = slice(e0, min(E, e0 + chunk))
            dj, ji = _flux_metrics(mesh, t, par.aa, sl)
            rt[sl] = _divergence(r, Up[t][sl], Q[t][sl], dj, ji, gas, par.aa, cast)
        Rt[t] = rt
    qfa = _flat(Qf, mesh, (3, 5))
    nL = cast(mesh.fnrm[mesh.iL])
    F = physics.common_normal_flux(uL.T, uR.T, qfa[mesh.iL].transpose(1, 2, 0),
                                   qfa[mesh.iR].transpose(1, 2, 0), nL.T, gas, beta, tau).T  # 11
    # the common normal flux is physical, equal and opposite on the two sides
    # (eq. FR-comm_flux); each side transforms it with its own area factor
    da = np.empty_like(ufa)
    da[mesh.iL] = cast(mesh.fmag[mesh.iL])[:, None] * F
    da[mesh.iR] = -(cast(mesh.fmag[mesh.iR])[:, None] * F)
    out = {}
    for t in mesh.types:
        r = mesh.refs[t]
        D = _unflat(da, mesh, t, (5,))
        rt = Rt[t] + np.einsum("uf,efv->euv", cast(r.M3), D)  # 12 tdivtconf
        du = -rt / _detj_u(mesh, t, None, cast)  # 13 negdivconf
        out[t] = du.transpose(0, 2, 1).copy()
    return out


def rk4_step(mesh, U, par, dt):
    """Classical four-stage Runge-Kutta step (the time integrator named in
    section 3); returns the new state."""
    def axpy(a, X, Y):
        return {t: Y[t] + a * X[t] for t in mesh.types}

    k1 = rhs(mesh, U, par)
    k2 = rhs(mesh, axpy(0.5 * dt, k1, U), par)
    k3 = rhs(mesh, axpy(0.5 * dt, k2, U), par)
    k4 = rhs(mesh, axpy(dt, k3, U), par)
    return {t: U[t] + (dt / 6.0) * (k1[t] + 2.0 * k2[t] + 2.0 * k3[t] + k4[t]) for t in mesh.types}


def rhs_subset(mesh, U, par, sel, dtype=None):
    """du = R(u) for selected elements only, with the same steps as rhs().

    sel: dict type -> array of element indices.  The RHS of an element needs
    the face states of its neighbours (for C and the common flux) and the
    gradients of its neighbours (for the common flux), which in turn need the
    face states of the neighbours' neighbours; so the disu step runs on the
    two-hop neighbourhood, con_u/gradients on the one-hop neighbourhood and
    the anti-aliased volume term only on the selected elements.  Returns
    dict type -> (len(sel[t]), 5, N_u)."""
    gas, beta, tau = par.gas, par.beta, par.tau
    if dtype is None:
        dtype = U[mesh.types[0]].dtype
    cast = lambda a: np.asarray(a, dtype=dtype)  # noqa: E731
    nt = len(mesh.types)
    ti = {t: i for i, t in enumerate(mesh.types)}

    def fpts_of(t, elems):
        r = mesh.refs[t]
        return (mesh.foff[t] + elems[:, None] * r.nf + np.arange(r.nf)[None, :]).reshape(-1)

    def neighbours(sets):
        out = [set(s) for s in sets]
        for t in mesh.types:
            idx = np.array(sorted(sets[ti[t]]), dtype=np.int64)
            if len(idx) == 0:
                continue
            pp = mesh.partner[fpts_of(t, idx)]
            for tt, ee in zip(mesh.ftype[pp], mesh.felem[pp]):
                out[tt].add(int(ee))
        return out

    S0 = [set(int(e) for e in sel.get(t, [])) for t in mesh.types]
    S1 = neighbours(S0)
    S2 = neighbours(S1)
    L0 = [np.array(sorted(s), dtype=np.int64) for s in S0]
    L1 = [np.array(sorted(s), dtype=np.int64) for s in S1]
    L2 = [np.array(sorted(s), dtype=np.int64) for s in S2]
    # flat flux point -> row in the compact S2 face arrays
    row = np.full(mesh.nfpts, -1, dtype=np.int64)
    blocks, off = [], 0
    Up = {}
    for t in mesh.types:
        r = mesh.refs[t]
        e2 = L2[ti[t]]
        fp = fpts_of(t, e2)
        row[fp] = off + np.arange(len(fp))
        off += len(fp)
        u = cast(U[t][e2]).transpose(0, 2, 1).copy()
        u[:, :, 4] -= cast(gas.eref)
        Up[t] = (e2, u)
        blocks.append(np.einsum("fu,euv->efv", cast(r.M0), u).reshape(-1, 5))  # 1 disu
    ufa = np.concatenate(blocks) if blocks else np.zeros((0, 5), dtype)
    Q, Qrow = {}, np.full(mesh.nfpts, -1, dtype=np.int64)
    qblocks, qoff = [], 0
    for t in mesh.types:
        r = mesh.refs[t]
        e1 = L1[ti[t]]
        if len(e1) == 0:
            continue
        e2, u2 = Up[t]
        pos = np.searchsorted(e2, e1)
        u = u2[pos]
        fp = fpts_of(t, e1)
        own = ufa[row[fp]].reshape(len(e1), r.nf, 5)
        nb = ufa[row[mesh.partner[fp]]].reshape(len(e1), r.nf, 5)
        left = np.zeros(mesh.nfpts, dtype=bool)
        left[mesh.iL] = True
        lf = left[fp].reshape(len(e1), r.nf, 1)
        C = np.where(lf, physics.common_solution(own, nb, beta), physics.common_solution(nb, own, beta))  # 2
        qt = np.einsum("dsu,euv->edsv", cast(r.Dg), u)  # 3
        qt += np.einsum("dsf,efv->edsv", cast(r.M6), C - own)  # 4
        q = _to_physical(mesh, t, qt, e1, cast)  # 5
        Q[t] = (e1, q)
        qblocks.append(np.einsum("fs,ecsv->efcv", cast(r.M0), q).reshape(-1, 3, 5))  # 6
        Qrow[fp] = qoff + np.arange(len(fp))
        qoff += len(fp)
    qfa = np.concatenate(qblocks)
    out = {}
    for t in mesh.types:
        r = mesh.refs[t]
        e0 = L0[ti[t]]
        if len(e0) == 0:
            continue
        e2, u2 = Up[t]
        u = u2[np.searchsorted(e2, e0)]
        e1, q1 = Q[t]
        q = q1[np.searchsorted(e1, e0)]
        dj, ji = _flux_metrics(mesh, t, par.aa, e0)
        rt = _divergence(r, u, q, dj, ji, gas, par.aa, cast)  # 7-10
        fp = fpts_of(t, e0)
        left = np.zeros(mesh.nfpts, dtype=bool)
        left[mesh.iL] = True
        lf = left[fp]
        pp = mesh.partner[fp]
        uo, un = ufa[row[fp]], ufa[row[pp]]
        qo, qn = qfa[Qrow[fp]], qfa[Qrow[pp]]
        iL = np.where(lf, fp, pp)
        nL = cast(mesh.fnrm[iL])
        uL, uR = np.where(lf[:, None], uo, un), np.where(lf[:, None], un, uo)
        qL, qR = np.where(lf[:, None, None], qo, qn), np.where(lf[:, None, None], qn, qo)
        F = physics.common_normal_flux(uL.T, uR.T, qL.transpose(1, 2, 0), qR.transpose(1, 2, 0), nL.T, gas, beta,
                                       tau).T  # 11
        mag = cast(mesh.fmag[fp])[:, None]  # own area factor (eq. FR-comm_flux)
        D = np.where(lf[:, None], mag * F, -(mag * F)).reshape(len(e0), r.nf, 5)
        rt = rt + np.einsum("uf,efv->euv", cast(r.M3), D)  # 12
        du = -rt / _detj_u(mesh, t, e0, cast)  # 13
        out[t] = du.transpose(0, 2, 1).copy()
    return out
