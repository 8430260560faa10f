"""Serving pool on the GPU (through the C ABI).

* the device Taylor-Green initial state equals the input generator's;
* a request run through the pool ends bit-identical to fr_rk4_step on the
  same mesh and state (same kernels, one launch over the batch);
* every request of a mixed batch (hex, prism and mixed meshes, orders 1-4,
  uneven sizes and step counts, admissions throttled by a small budget and
  slot limit) ends bit-identical to the same request run alone;
* a pool result matches the oracle's RK4 within the FP64 tolerance.
"""

import numpy as np
import pytest

import paper_2401_06132_amd as frmi
from oracle.mesh import Mesh
from oracle.rhs import Params, rk4_step as oracle_rk4
from paper_2401_06132_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _init(n, p, kind, seed):
    s = frmi.Solver(n, p, kind)
    U = inputs.element_state(s.upts_coords(), seed=seed)
    return np.concatenate([u.reshape(-1) for u in U])


def _drain(pool, budget=None, max_active=None):
    rounds = 0
    while True:
        st, _, _ = pool.step()
        if budget is not None:
            assert st["bytes_in_use"] <= budget
        if max_active is not None:
            assert st["n_active"] <= max_active
        rounds += 1
        if st["n_active"] == 0 and st["n_queued"] == 0 and st["n_admitted"] == 0:
            return rounds
        assert rounds < 10000


@pytest.mark.parametrize("kind,n,p", [("hex", 3, 3), ("prism", 3, 2), ("mixed", 4, 4)])
def test_pool_tgv_initial_state(kind, n, p):
    _need_gpu()
    print("pool tgv init", kind, n, p, flush=True)
    pool = frmi.Pool(1 << 28, prec="fp64", pref=inputs.P0, rho_ref=inputs.RHO0)
    _, ns = pool.footprint(n=n, p=p, kind=kind, tgv_p0=inputs.P0)
    out = np.full(ns, np.nan)
    pool.submit(n=n, p=p, kind=kind, nsteps=0, tgv_p0=inputs.P0, u_out=out)
    _drain(pool)
    s = frmi.Solver(n, p, kind)
    ref = np.concatenate([np.ascontiguousarray(inputs.tgv_state(c).transpose(0, 2, 1)).reshape(-1)
                          for c in s.upts_coords()])
    assert np.allclose(out, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind,n,p", [("hex", (3, 2, 4), 2), ("prism", 3, 3), ("mixed", 4, 1)])
def test_pool_equals_rk4_step(kind, n, p, prec):
    _need_gpu()
    print("pool vs rk4", kind, n, p, prec, flush=True)
    u0 = _init(n, p, kind, seed=3)
    dt, steps = 2e-4, 5
    s = frmi.Solver(n, p, kind, prec=prec, pref=inputs.P0, rho_ref=inputs.RHO0)
    s.set_state(u0)
    s.rk4(dt, steps)
    ref = s.get_state()
    pool = frmi.Pool(1 << 28, prec=prec, pref=inputs.P0, rho_ref=inputs.RHO0)
    out = np.empty_like(u0)
    pool.submit(n=n, p=p, kind=kind, nsteps=steps, dt=dt, u_init=u0, u_out=out)
    _drain(pool)
    assert np.array_equal(out, ref)


def _mix():
    # (n, p, kind, steps): uneven sizes, all element kinds, orders 1-4
    return [((4, 3, 5), 2, "hex", 7), (3, 3, "prism", 3), (4, 4, "mixed", 5), (2, 1, "hex", 9),
            ((2, 3, 2), 4, "prism", 4), (5, 2, "hex", 2), (3, 3, "hex", 6), (4, 2, "mixed", 3),
            (3, 4, "hex", 4), (2, 3, "prism", 8)]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_pool_solo_equals_batched(prec):
    """Each request alone and in the mix ends with the same bits (the stated
    tolerance is met trivially: the per-element arithmetic does not depend on
    the batch)."""
    _need_gpu()
    mix = _mix()
    dt = 1e-4
    inits = [_init(n, p, kind, seed=10 + i) for i, (n, p, kind, _) in enumerate(mix)]
    solo = []
    for i, ((n, p, kind, steps), u0) in enumerate(zip(mix, inits)):
        print("solo", i, n, p, kind, steps, prec, flush=True)
        pool = frmi.Pool(1 << 28, prec=prec, pref=inputs.P0, rho_ref=inputs.RHO0)
        out = np.empty_like(u0)
        pool.submit(n=n, p=p, kind=kind, nsteps=steps, dt=dt, u_init=u0, u_out=out)
        _drain(pool)
        solo.append(out)
    # batched: a budget that holds about a third of the mix and 4 slots, so
    # requests queue and are admitted as others finish; half the requests are
    # submitted after the first rounds (arrivals while others run)
    pool = frmi.Pool(1 << 28, prec=prec, pref=inputs.P0, rho_ref=inputs.RHO0)
    fp = [pool.footprint(n=n, p=p, kind=kind, tgv_p0=1.0)[0] for n, p, kind, _ in mix]
    budget = max(max(fp), sum(fp) // 3)
    max_active = 4
    print("batched", prec, "budget", budget, flush=True)
    pool = frmi.Pool(budget, max_active=max_active, prec=prec, pref=inputs.P0, rho_ref=inputs.RHO0)
    outs = [np.full_like(u, np.nan) for u in inits]
    half = len(mix) // 2
    for i in range(half):
        n, p, kind, steps = mix[i]
        pool.submit(n=n, p=p, kind=kind, nsteps=steps, dt=dt, u_init=inits[i], u_out=outs[i])
    for _ in range(3):
        st, _, _ = pool.step()
        assert st["bytes_in_use"] <= budget and st["n_active"] <= max_active
    for i in range(half, len(mix)):
        n, p, kind, steps = mix[i]
        pool.submit(n=n, p=p, kind=kind, nsteps=steps, dt=dt, u_init=inits[i], u_out=outs[i])
    _drain(pool, budget=budget, max_active=max_active)
    for i, (a, b) in enumerate(zip(solo, outs)):
        assert np.array_equal(a, b), i


def test_pool_matches_oracle():
    """A pool request (FP64, mixed mesh, 3 RK4 steps) against the oracle's
    RK4, on the state change; same bar as the single-context RK4 test."""
    _need_gpu()
    dims, p, steps, dt = (2, 2, 4), 2, 3, 1e-3
    m = Mesh(*dims, p, "mixed")
    U = inputs.element_state([m.upts_coords(t) for t in m.types], seed=5)
    par = Params(pref=inputs.P0)
    Uo = dict(zip(m.types, U))
    for _ in range(steps):
        Uo = oracle_rk4(m, Uo, par, dt)
    u0 = np.concatenate([u.reshape(-1) for u in U])
    pool = frmi.Pool(1 << 28, prec="fp64", pref=inputs.P0, rho_ref=inputs.RHO0)
    out = np.empty_like(u0)
    pool.submit(n=dims, p=p, kind="mixed", nsteps=steps, dt=dt, u_init=u0, u_out=out)
    _drain(pool)
    s = frmi.Solver(dims, p, "mixed")
    got = s.split(out)
    for t, g, u in zip(m.types, got, U):
        d_ref = Uo[t] - u
        err = np.abs((g - u) - d_ref).max(axis=(0, 2)) / np.abs(d_ref).max(axis=(0, 2))
        print("pool vs oracle", t, err)
        assert np.all(err < 1e-11)


@pytest.mark.parametrize("kind", ["hex", "mixed"])
def test_pool_without_anti_aliasing_equals_rk4_step(kind):
    """A pool in the configuration without flux anti-aliasing ends
    bit-identical to fr_rk4_step in the same configuration."""
    _need_gpu()
    n, p, steps, dt = (3, 2, 4), 3, 4, 2e-4
    u0 = _init(n, p, kind, seed=4)
    s = frmi.Solver(n, p, kind, prec="fp32", pref=inputs.P0, rho_ref=inputs.RHO0, aa=False)
    s.set_state(u0)
    s.rk4(dt, steps)
    ref = s.get_state()
    pool = frmi.Pool(1 << 28, prec="fp32", pref=inputs.P0, rho_ref=inputs.RHO0, aa=False)
    out = np.empty_like(u0)
    pool.submit(n=n, p=p, kind=kind, nsteps=steps, dt=dt, u_init=u0, u_out=out)
    _drain(pool)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("kind", ["hex", "prism", "mixed"])
def test_pool_full_anti_aliasing_equals_rk4_step(kind):
    """A pool with flux and surface-flux anti-aliasing (the surface kernels
    then run half the elements per workgroup) ends bit-identical to
    fr_rk4_step in the same configuration, also batched with a second
    request of another order."""
    _need_gpu()
    n, p, steps, dt = (3, 2, 4), 3, 4, 2e-4
    u0 = _init(n, p, kind, seed=5)
    s = frmi.Solver(n, p, kind, prec="fp32", pref=inputs.P0, rho_ref=inputs.RHO0, surface_aa=True)
    s.set_state(u0)
    s.rk4(dt, steps)
    ref = s.get_state()
    pool = frmi.Pool(1 << 28, prec="fp32", pref=inputs.P0, rho_ref=inputs.RHO0, surface_aa=True)
    out = np.empty_like(u0)
    pool.submit(n=n, p=p, kind=kind, nsteps=steps, dt=dt, u_init=u0, u_out=out)
    pool.submit(n=(2, 3, 2), p=2, kind="prism", nsteps=3, dt=dt, tgv_p0=inputs.P0)
    _drain(pool)
    assert np.array_equal(out, ref)


def test_pool_failed_admission_does_not_disturb_the_round():
    """A request whose host set-up fails (injected) leaves the queue as
    failed; the requests admitted beside it and the ones already running
    take exactly their own steps and end bit-identical to fr_rk4_step."""
    _need_gpu()
    print("pool failed admission", flush=True)
    n, p, kind, dt = 3, 2, "hex", 2e-4
    u0 = _init(n, p, kind, seed=5)
    pool = frmi.Pool(1 << 28, max_active=4, prec="fp64", pref=inputs.P0, rho_ref=inputs.RHO0)
    outs, steps = {}, {}
    first = pool.submit(n=n, p=p, kind=kind, nsteps=4, dt=dt, u_init=u0, u_out=np.empty_like(u0))
    outs[first], steps[first] = pool._keep[first][1], 4
    pool.step()  # the first request is admitted and runs from the next round
    bad = pool.submit(n=n, p=p, kind=kind, nsteps=3, dt=dt, u_init=u0)
    pool.inject_prepare_error(bad)
    last = pool.submit(n=n, p=p, kind=kind, nsteps=2, dt=dt, u_init=u0, u_out=np.empty_like(u0))
    outs[last], steps[last] = pool._keep[last][1], 2
    finished = []
    for _ in range(100):
        st, _, fin = pool.step()
        finished += fin
        if st["n_active"] == 0 and st["n_queued"] == 0 and st["n_admitted"] == 0:
            break
    assert bad in finished and pool.query(bad) == (frmi.Pool.FAILED, 0)
    for rid, out in outs.items():
        assert pool.query(rid) == (frmi.Pool.DONE, steps[rid])
        s = frmi.Solver(n, p, kind, prec="fp64", pref=inputs.P0, rho_ref=inputs.RHO0)
        s.set_state(u0)
        s.rk4(dt, steps[rid])
        assert np.array_equal(out, s.get_state())
