"""Host-side checks of the serving pool (no GPU: creation, footprints and
submission make no device call)."""

import numpy as np
import pytest

import paper_2401_06132_amd as frmi


def _expected_bytes(n, p, kind, rs):
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    h = -np.pi + (np.arange(nz) + 0.5) * (2 * np.pi / nz)
    hexcells = nx * ny * (nz if kind == "hex" else (0 if kind == "prism" else int(np.sum(h < 0))))
    ne = [hexcells, 2 * (nx * ny * nz - hexcells)]
    k = p + 1
    nu = [k ** 3, k * k * (k + 1) // 2]
    ns = 5 * (ne[0] * nu[0] + ne[1] * nu[1])
    slots = 6 * ne[0] + 5 * ne[1]
    pts = 6 * k * k * ne[0] + (k * (k + 1) + 3 * k * k) * ne[1]  # quadrilateral and triangle faces
    parts = [8 * ns, 8 * ns, 8 * ns, rs * ns, rs * 5 * pts, rs * 4 * pts, 16 * slots,
             rs * 4 * slots, 16 * k * k]
    if rs == 4:
        parts.append(4 * 5 * slots)  # single precision: one float base per face and variable
    for t in range(2):
        parts += [rs * 10 * ne[t], 8 * ne[t]]
    return sum(al(x) for x in parts), ns


@pytest.mark.parametrize("prec,rs", [("fp64", 8), ("fp32", 4)])
@pytest.mark.parametrize("n,p,kind", [(6, 2, "hex"), (7, 3, "prism"), ((5, 4, 6), 4, "mixed"), (32, 4, "prism"),
                                      (1, 1, "hex")])
def test_footprint(n, p, kind, prec, rs):
    pool = frmi.Pool(1 << 40, prec=prec)
    b, ns = pool.footprint(n=n, p=p, kind=kind, tgv_p0=1.0)
    eb, ens = _expected_bytes(n, p, kind, rs)
    assert (b, ns) == (eb, ens)
    s = frmi.Solver(n, p, kind)
    assert ns == s.n_state


def test_submit_validation_and_queue():
    pool = frmi.Pool(64 << 20, max_active=2, prec="fp32")
    with pytest.raises(frmi.FrError, match="FR_EINVAL"):
        pool.submit(n=4, p=2, kind="hex", nsteps=1)              # no initial state
    with pytest.raises(frmi.FrError, match="FR_EUNSUPPORTED"):
        pool.submit(n=4, p=5, kind="hex", nsteps=1, tgv_p0=1.0)  # order
    with pytest.raises(frmi.FrError, match="FR_EINVAL"):
        pool.submit(n=4, p=2, kind="hex", nsteps=-1, tgv_p0=1.0)
    with pytest.raises(frmi.FrError, match="FR_ENOMEM"):
        pool.submit(n=32, p=4, kind="prism", nsteps=1, tgv_p0=1.0)  # above the whole budget
    with pytest.raises(frmi.FrError):
        pool.submit(n=4, p=2, kind="hex", nsteps=1, u_init=np.zeros(3))  # wrong size
    ids = [pool.submit(n=4, p=2, kind="hex", nsteps=3, tgv_p0=1.0) for _ in range(3)]
    assert ids == [0, 1, 2]
    assert all(pool.query(i) == (frmi.Pool.QUEUED, 0) for i in ids)
    with pytest.raises(frmi.FrError):
        pool.query(99)


def test_plain_form_rejected():
    with pytest.raises(frmi.FrError, match="FR_EUNSUPPORTED"):
        lib = frmi.load_library()
        import ctypes
        ph = frmi.physics(form="plain")
        c = ctypes.c_void_p()
        frmi._check(None, lib.fr_pool_create(ctypes.byref(ph), None, 1 << 20, 4, ctypes.byref(c)))


def test_preparation_worker_starts_and_joins():
    """Submitting starts the host preparation worker (mesh and connectivity
    of the next queued requests, no device call); destroying the pool stops
    and joins it, also while a build is in flight."""
    import time
    for wait in (0.0, 0.3):
        pool = frmi.Pool(4 << 30, max_active=2, prec="fp64")
        for n, p, kind in [(4, 2, "hex"), (6, 3, "prism"), (24, 4, "prism"), (3, 1, "mixed"), (5, 2, "hex")]:
            pool.submit(n=n, p=p, kind=kind, nsteps=2, tgv_p0=1.0)
        time.sleep(wait)
        del pool


def test_failed_preparation_leaves_the_queue():
    """A request whose host set-up fails leaves the queue as failed before
    any device work of the round, and the requests behind it stay queued.
    Here the round's device work then fails for want of a GPU (or runs, on
    a GPU machine); the request states are what is checked."""
    import time

    pool = frmi.Pool(64 << 20, max_active=4, prec="fp64")
    ids = [pool.submit(n=3, p=2, kind="hex", nsteps=2, tgv_p0=1.0) for _ in range(3)]
    pool.inject_prepare_error(ids[0])
    with pytest.raises(frmi.FrError, match="FR_EINVAL"):
        pool.inject_prepare_error(99)
    for _ in range(200):  # until the preparation worker has reached request 0
        try:
            pool.step()
        except frmi.FrError:
            pass
        if pool.query(ids[0])[0] == frmi.Pool.FAILED:
            break
        time.sleep(0.01)
    assert pool.query(ids[0]) == (frmi.Pool.FAILED, 0)
    assert pool.query(ids[1])[0] in (frmi.Pool.QUEUED, frmi.Pool.ACTIVE)
    with pytest.raises(frmi.FrError, match="FR_EINVAL"):
        pool.inject_prepare_error(ids[0])  # no longer queued
