"""A NumPy emulation of the single-precision RHS as the fused kernels split
it, on a sampled subset of a mesh.  Test infrastructure: it uses the
oracle's meshes and dense operators (the kernels factorise them), and rounds
every intermediate the way the kernels do, so that the floor of a precision
split can be measured on the CPU.

Two splits, selected by `split`:
  "kernels" -- the split of the fused kernels:
      * the state in double precision relative to the reference state
        (rho' = rho - rho0, E' = E - pref/(gamma-1)), then rounded;
      * face values interpolated in double and stored per face as a
        single-precision base (the value at the face's first flux point)
        plus single-precision deviations, so face jumps are formed as
        (b_nbr - b_own) + (d_nbr - d_own);
      * gradients, anti-aliased fluxes and their weak-form divergence in
        single precision, with the energy flux split exactly as
        v (E + p) = v (E' + p' - kap rho') + kap rho v, kap = href / rho0;
      * L(rho v) = sum_d D_d (S m)_d in double: the mass residual, and kap
        times it in the energy residual; at the interface the strong-form
        term 1/2 (m_nbr - m_own) . n_own of both;
      * volume residual plus lifted interface flux summed in single
        precision, divided by det J in double.
  "energy_shift" -- the earlier split: only E is shifted, everything after
      the shift (face values, jumps, all five fluxes) in single precision.
With dtype float64 the "kernels" split is the RHS itself, rearranged: it
must agree with the oracle to rounding, which pins the algebra of the split.
Single mesh type, affine elements (hexahedra or prisms)."""

import numpy as np

from oracle import basis
from oracle.rhs import _flux_metrics, _to_physical


def _prim(u, gas, rho0):
    rho = u[0] + rho0
    v = u[1:4] / rho
    pp = (gas.gamma - 1) * (u[4] - 0.5 * np.sum(u[1:4] * v, axis=0))
    return rho, v, pp


def _inviscid(u, gas, rho0, kap, R):
    """f^e (3, 5, ...) in reference-state form; the energy component split
    (H = E' + p' + hc0 - kap rho')."""
    rho, v, pp = _prim(u, gas, rho0)
    hc0 = R(0) if kap else R(gas.href)
    h = u[4] + pp + hc0 - R(kap) * u[0]
    f = np.empty((3,) + u.shape, dtype=u.dtype)
    for d in range(3):
        f[d, 0] = u[1 + d]
        for i in range(3):
            f[d, 1 + i] = u[1 + d] * v[i]
        f[d, 1 + d] += pp
        f[d, 4] = v[d] * h
    return f


def _viscous(u, q, gas, rho0, R):
    mu = R(gas.mu)
    rho, v, _ = _prim(u, gas, rho0)
    gv = (q[:, 1:4] - v[None, :] * q[:, 0][:, None]) / rho
    div = gv[0, 0] + gv[1, 1] + gv[2, 2]
    etot = u[4] + R(gas.eref)
    ge = (q[:, 4] - (etot / rho) * q[:, 0]) / rho - np.sum(v[None, :] * gv, axis=1)
    f = np.zeros((3,) + u.shape, dtype=u.dtype)
    for d in range(3):
        for i in range(3):
            t = mu * (gv[d, i] + gv[i, d])
            if i == d:
                t = t - R(2.0 / 3.0) * mu * div
            f[d, 1 + i] = t
        f[d, 4] = sum(v[i] * f[d, 1 + i] for i in range(3)) + R(gas.mu * gas.gamma / gas.prandtl) * ge[d]
    return f


def _weak_divergence(r):
    """AP_d = -Mass^-1 Dq_d^T W_q (3, N_u, N_q): the weak form that the
    kernels apply for (M1 - M3 M2) M9."""
    _, Dq = basis.nodal(r.etype, r.p, r.upts, r.qpts)
    minv = basis.inv(r.mass)
    w = np.asarray(r.qwts, dtype=basis.EXT)
    return np.stack([-(minv @ (Dq[d].T * w[None, :])) for d in range(3)]).astype(np.float64)


def rhs_split(mesh, U, par, sel, dtype=np.float32, split="kernels", rho0=1.0):
    """du of the selected elements, (len(sel), 5, N_u) float64."""
    R = dtype
    cast = lambda a: np.asarray(a, dtype=R)  # noqa: E731
    gas, beta, tau = par.gas, par.beta, par.tau
    t = mesh.types[0]
    assert len(mesh.types) == 1 and not mesh.curved
    r = mesh.refs[t]
    new = split == "kernels"
    r0 = rho0 if new else 0.0
    kap = gas.href / rho0 if new else 0.0
    R0 = R(r0)

    def fpts_of(elems):
        return (mesh.foff[t] + elems[:, None] * r.nf + np.arange(r.nf)[None, :]).reshape(-1)

    def hop(s):
        return set(s) | set(int(e) for e in mesh.felem[mesh.partner[fpts_of(np.array(sorted(s)))]])

    S0 = set(int(e) for e in sel)
    S1 = hop(S0)
    L0, L1, L2 = [np.array(sorted(x)) for x in (S0, S1, hop(S1))]
    row = np.full(mesh.nfpts, -1, dtype=np.int64)
    row[fpts_of(L2)] = np.arange(len(L2) * r.nf)
    u64 = U[L2].transpose(0, 2, 1).copy()  # (E, N_u, 5)
    u64[:, :, 4] -= gas.eref
    u64[:, :, 0] -= r0
    u32 = cast(u64)
    # face values: base + deviations (kernels), or single precision throughout
    if new:
        f64 = np.einsum("fu,euv->efv", r.M0, u64)
        bas = np.zeros(f64.shape, dtype=R)
        for fi in range(r.nfaces):
            cols = np.nonzero(r.fface == fi)[0]
            bas[:, cols, :] = cast(f64[:, cols[0], :])[:, None, :]
        dev = cast(f64 - bas.astype(np.float64))
    else:
        dev = np.einsum("fu,euv->efv", cast(r.M0), u32)
        bas = np.zeros_like(dev)
    bas, dev = bas.reshape(-1, 5), dev.reshape(-1, 5)

    def val(i):
        return bas[i] + dev[i]

    def jump(a, b):  # value(a) - value(b)
        return (bas[a] - bas[b]) + (dev[a] - dev[b])

    left = np.zeros(mesh.nfpts, dtype=bool)
    left[mesh.iL] = True
    # corrected gradients on the one-hop neighbourhood
    u1 = u32[np.searchsorted(L2, L1)]
    fp1 = fpts_of(L1)
    own = np.einsum("fu,euv->efv", cast(r.M0), u1)
    nbv = val(row[mesh.partner[fp1]]).reshape(len(L1), r.nf, 5)
    lf1 = left[fp1].reshape(len(L1), r.nf, 1)
    jm = np.where(lf1, R(0.5 + beta), R(0.5 - beta)) * (nbv - own)
    qt = np.einsum("dsu,euv->edsv", cast(r.Dg), u1) + np.einsum("dsf,efv->edsv", cast(r.M6), jm)
    q1 = _to_physical(mesh, t, qt, L1, cast)
    qfa = np.einsum("fs,ecsv->efcv", cast(r.M0), q1).reshape(-1, 3, 5)
    qrow = np.full(mesh.nfpts, -1, dtype=np.int64)
    qrow[fp1] = np.arange(len(fp1))
    # anti-aliased volume term (weak form) on the selected elements
    pos0 = np.searchsorted(L2, L0)
    u0, q0 = u32[pos0], q1[np.searchsorted(L1, L0)]
    dj, ji = _flux_metrics(mesh, t, par.aa, L0)
    uq = np.einsum("qu,euv->vqe", cast(r.M7), u0)
    qq = np.einsum("qs,ecsv->cvqe", cast(r.M7), q0)
    f = _inviscid(uq, gas, R0, kap, R) - _viscous(uq, qq, gas, R0, R)
    ft = np.einsum("e,edc,cvqe->edqv", cast(dj), cast(ji), f)
    rt = np.einsum("dsq,edqv->esv", cast(_weak_divergence(r)), ft)
    if new:
        # L(rho v) in double: the mass residual and kap times it in energy
        sm = np.einsum("e,edc,euc->edu", mesh.detJ[t][L0], mesh.Jinv[t][L0], u64[pos0][:, :, 1:4])
        lv = cast(np.einsum("dsu,edu->es", r.Dg, sm))
        rt[:, :, 0] = lv
        rt[:, :, 4] += R(kap) * lv
    # interface flux at the own flux points
    fp0 = fpts_of(L0)
    lf0 = left[fp0]
    io, ino = row[fp0], row[mesh.partner[fp0]]
    iL = np.where(lf0, fp0, mesh.partner[fp0])
    nL = cast(mesh.fnrm[iL]).T
    iLr, iRr = np.where(lf0, io, ino), np.where(lf0, ino, io)
    uL, uR, jLR = val(iLr).T, val(iRr).T, jump(iLr, iRr).T
    qo, qn = qfa[qrow[fp0]], qfa[qrow[mesh.partner[fp0]]]
    qL = np.where(lf0[:, None, None], qo, qn).transpose(1, 2, 0)
    qR = np.where(lf0[:, None, None], qn, qo).transpose(1, 2, 0)
    feL, feR = _inviscid(uL, gas, R0, kap, R), _inviscid(uR, gas, R0, kap, R)
    fvL, fvR = _viscous(uL, qL, gas, R0, R), _viscous(uR, qR, gas, R0, R)
    _, vL, pL = _prim(uL, gas, R0)
    _, vR, pR = _prim(uR, gas, R0)
    cL = np.sqrt(R(gas.gamma) * (pL + R(gas.pref)) / (uL[0] + R0))
    cR = np.sqrt(R(gas.gamma) * (pR + R(gas.pref)) / (uR[0] + R0))
    s = np.maximum(np.abs(np.sum(vL * nL, 0)) + cL, np.abs(np.sum(vR * nL, 0)) + cR)
    a = R(0.5) * s + R(tau)
    F = R(0.5) * np.einsum("dvp,dp->vp", feL + feR, nL) + a * jLR
    F -= np.einsum("dvp,dp->vp", R(0.5 + beta) * fvL + R(0.5 - beta) * fvR, nL)
    mag = cast(mesh.fmag[fp0])
    sg = np.where(lf0, R(1), R(-1))
    D = (sg * mag * F).T
    if new:
        jn = jump(ino, io)[:, 1:4]  # m_nbr - m_own
        half = R(0.5) * mag * np.sum(jn * (sg * nL).T, axis=1)
        D[:, 0] = half - mag * a * jump(ino, io)[:, 0]
        D[:, 4] += R(kap) * half
    lift = np.einsum("uf,efv->euv", cast(r.M3), D.reshape(len(L0), r.nf, 5))
    du = -(rt + lift).astype(np.float64) / mesh.detJ[t][L0][:, None, None]
    return du.transpose(0, 2, 1)
