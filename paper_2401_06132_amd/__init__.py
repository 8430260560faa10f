"""MI355X flux-reconstruction library: Python binding of libfrmi.so.

Thin ctypes wrapper over the C ABI declared in include/fr.h: argument
marshalling only.  Every step of the right-hand side and of RK4 runs in the
HIP kernels of the shared library; there is no fallback.  Device buffers are
torch tensors (float64, on the current HIP device); PyTorch is used for
device memory and streams only.
"""

import ctypes
import os

import numpy as np

from . import inputs  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfrmi.so")

FR_HEX, FR_PRISM = 0, 1
MESH_KIND = {"hex": 0, "prism": 1, "mixed": 2, "tet": 3, "prism_tet": 4, "hex_warp": 5, "prism_warp": 6,
             "mixed_warp": 7, "pyr": 8, "hex_pyr": 9, "hex_pyr_tet": 10,
             "hex_prism_pyr_tet": 11}
PREC = {"fp64": 0, "fp32": 1}
FORM = {"fused": 0, "plain": 1}
_STATUS = {0: "FR_OK", -1: "FR_EINVAL", -2: "FR_ENOMEM", -3: "FR_EDEVICE", -4: "FR_ESTATE", -5: "FR_EUNSUPPORTED"}

# every symbol the header declares
SYMBOLS = ["fr_physics_default", "fr_create", "fr_mesh_box", "fr_mesh_elements", "fr_layout", "fr_type_count", "fr_upts_coords", "fr_rhs",
           "fr_rhs_noalloc", "fr_rhs_stages", "fr_set_state", "fr_get_state", "fr_rk4_step", "fr_integrals", "fr_ref_operator", "fr_connectivity",
           "fr_last_error", "fr_destroy", "fr_fill_lds", "fr_pool_create", "fr_pool_footprint", "fr_pool_submit", "fr_pool_step",
           "fr_pool_events", "fr_pool_query", "fr_pool_inject_prepare_error", "fr_pool_last_error", "fr_pool_destroy"]


class FrPhysics(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("prandtl", ctypes.c_double), ("mu", ctypes.c_double),
                ("ldg_beta", ctypes.c_double), ("ldg_tau", ctypes.c_double), ("pref", ctypes.c_double),
                ("rho_ref", ctypes.c_double), ("prec", ctypes.c_int), ("form", ctypes.c_int), ("flux_aa", ctypes.c_int),
                ("surface_aa", ctypes.c_int)]


class FrRequest(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("lo", ctypes.c_double),
                ("hi", ctypes.c_double), ("p", ctypes.c_int), ("kind", ctypes.c_int), ("dt", ctypes.c_double),
                ("nsteps", ctypes.c_int), ("u_init", ctypes.c_void_p), ("tgv_p0", ctypes.c_double),
                ("u_out", ctypes.c_void_p)]


class FrPoolStats(ctypes.Structure):
    _fields_ = [("n_active", ctypes.c_int), ("n_admitted", ctypes.c_int), ("n_finished", ctypes.c_int),
                ("n_queued", ctypes.c_int), ("n_launches", ctypes.c_int), ("dof", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_int64)]


class FrError(RuntimeError):
    pass


_lib = None


def load_library(path=None):
    """Load libfrmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise FrError("libfrmi.so not built; run paper_2401_06132_amd.build.build()")
    try:
        # torch ships its own HIP runtime; loaded first, it is the one the
        # library binds to as well, so both share one runtime and device
        # pointers pass between them.  Loaded after the library, a second
        # runtime would come up beside the first and see no device.
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sig = {
        "fr_physics_default": (None, [ctypes.POINTER(FrPhysics)]),
        "fr_create": (I, [ctypes.POINTER(FrPhysics), P, ctypes.POINTER(P)]),
        "fr_mesh_box": (I, [P, I, I, I, D, D, I, I]),
        "fr_mesh_elements": (I, [P, I, P, P, P]),
        "fr_layout": (I, [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64)]),
        "fr_type_count": (I, [P, I, ctypes.POINTER(I64)]),
        "fr_upts_coords": (I, [P, P]),
        "fr_rhs": (I, [P, P, P]),
        "fr_rhs_noalloc": (I, [P, P, P]),
        "fr_rhs_stages": (I, [P, P, P, I]),
        "fr_set_state": (I, [P, P, I]),
        "fr_get_state": (I, [P, P, I]),
        "fr_rk4_step": (I, [P, D, I]),
        "fr_integrals": (I, [P, P]),
        "fr_ref_operator": (I, [I, I, ctypes.c_char_p, P, I64, ctypes.POINTER(I64)]),
        "fr_connectivity": (I, [P, P, P, ctypes.POINTER(I64)]),
        "fr_last_error": (ctypes.c_char_p, [P]),
        "fr_destroy": (None, [P]),
        "fr_fill_lds": (I, [P, ctypes.c_float]),
        "fr_pool_create": (I, [ctypes.POINTER(FrPhysics), P, I64, I, ctypes.POINTER(P)]),
        "fr_pool_footprint": (I, [P, ctypes.POINTER(FrRequest), ctypes.POINTER(I64), ctypes.POINTER(I64)]),
        "fr_pool_submit": (I, [P, ctypes.POINTER(FrRequest), ctypes.POINTER(I64)]),
        "fr_pool_step": (I, [P, ctypes.POINTER(FrPoolStats)]),
        "fr_pool_events": (I, [P, P, ctypes.POINTER(I), P, ctypes.POINTER(I), I]),
        "fr_pool_query": (I, [P, I64, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "fr_pool_inject_prepare_error": (I, [P, I64]),
        "fr_pool_last_error": (ctypes.c_char_p, [P]),
        "fr_pool_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def physics(gamma=1.4, prandtl=0.71, mu=1.0 / 1600.0, beta=0.5, tau=0.1, pref=0.0, rho_ref=0.0, prec="fp64",
            form="fused", aa=True, surface_aa=False):
    """pref, rho_ref: reference pressure and density of the reference-state
    form; aa: flux anti-aliasing; surface_aa: surface-flux anti-aliasing as
    well (the paper's "full AA" with aa=True)."""
    return FrPhysics(gamma, prandtl, mu, beta, tau, pref, rho_ref, PREC[prec], FORM[form], 1 if aa else 0,
                     1 if surface_aa else 0)


def ref_operator(etype, p, name):
    """Reference-element quantity computed by the library's host setup."""
    lib = load_library()
    cnt = ctypes.c_int64(0)
    _check(None, lib.fr_ref_operator(etype, p, name.encode(), None, 0, ctypes.byref(cnt)))
    out = np.empty(cnt.value, dtype=np.float64)
    _check(None, lib.fr_ref_operator(etype, p, name.encode(), out.ctypes.data, cnt.value, ctypes.byref(cnt)))
    return out


def fill_lds(value, stream=None):
    """Fill the device's LDS with `value` (asynchronous on the HIP stream
    handle `stream`, default the null stream).  Test support: running the
    kernels after a fill with NaN shows that none reads LDS it has not
    written."""
    lib = load_library()
    _check(None, lib.fr_fill_lds(stream, float(value)))


def _check(ctx, st, pool=False):
    if st != 0:
        lib = load_library()
        msg = (lib.fr_pool_last_error(ctx) if pool else lib.fr_last_error(ctx)).decode() if ctx else ""
        raise FrError("%s: %s" % (_STATUS.get(st, st), msg))


class Solver:
    """One flux-reconstruction context (mesh + operators + device buffers)."""

    def __init__(self, n, p, kind="hex", prec="fp64", form="fused", lo=-np.pi, hi=np.pi, stream=None, verts=None,
                 period=None, **phys):
        """A periodic box (n cells per axis, or (nx, ny, nz), of mesh kind
        `kind`), or with kind="elements" a general affine mesh: verts = dict
        type name -> (E, nv, 3) vertex array (hex, prism, tet, pyr; vertex
        orders as in fr_mesh_elements), period = (3, 3) period vectors or
        None."""
        self.lib = load_library()
        ph = physics(prec=prec, form=form, **phys)
        c = ctypes.c_void_p()
        st = None if stream is None else ctypes.c_void_p(stream)
        _check(None, self.lib.fr_create(ctypes.byref(ph), st, ctypes.byref(c)))
        self.ctx = c
        self.p, self.kind, self.prec = p, kind, prec
        if kind == "elements":
            names = ("hex", "prism", "tet", "pyr")
            arrs = [np.ascontiguousarray(verts[t], dtype=np.float64) if t in verts else None for t in names]
            counts = (ctypes.c_int64 * 4)(*[0 if a is None else a.shape[0] for a in arrs])
            ptrs = (ctypes.c_void_p * 4)(*[None if a is None else a.ctypes.data for a in arrs])
            per = None if period is None else np.ascontiguousarray(period, dtype=np.float64).reshape(9)
            _check(self.ctx, self.lib.fr_mesh_elements(self.ctx, p, counts, ptrs,
                                                       None if per is None else per.ctypes.data))
        else:
            nx, ny, nz = (n, n, n) if np.isscalar(n) else n
            _check(self.ctx, self.lib.fr_mesh_box(self.ctx, nx, ny, nz, lo, hi, p, MESH_KIND[kind]))
        nh, npr, ns = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(self.ctx, self.lib.fr_layout(self.ctx, ctypes.byref(nh), ctypes.byref(npr), ctypes.byref(ns)))
        self.n_hex, self.n_prism, self.n_state = nh.value, npr.value, ns.value
        nt, npy = ctypes.c_int64(), ctypes.c_int64()
        _check(self.ctx, self.lib.fr_type_count(self.ctx, 2, ctypes.byref(nt)))
        _check(self.ctx, self.lib.fr_type_count(self.ctx, 3, ctypes.byref(npy)))
        self.n_tet, self.n_pyr = nt.value, npy.value
        n1 = p + 1
        self.nu = {"hex": n1 ** 3, "prism": (n1 * (n1 + 1) // 2) * n1, "tet": n1 * (n1 + 1) * (n1 + 2) // 6,
                   "pyr": n1 * (n1 + 1) * (2 * n1 + 1) // 6}

    def __del__(self):
        if getattr(self, "ctx", None):
            self.lib.fr_destroy(self.ctx)
            self.ctx = None

    @property
    def n_dof(self):
        return self.n_state

    def blocks(self):
        """[(type name, element count, points per element)] in library order."""
        out = []
        if self.n_hex:
            out.append(("hex", self.n_hex, self.nu["hex"]))
        if self.n_prism:
            out.append(("prism", self.n_prism, self.nu["prism"]))
        if self.n_tet:
            out.append(("tet", self.n_tet, self.nu["tet"]))
        if self.n_pyr:
            out.append(("pyr", self.n_pyr, self.nu["pyr"]))
        return out

    def upts_coords(self):
        xyz = np.empty((self.n_state // 5, 3))
        _check(self.ctx, self.lib.fr_upts_coords(self.ctx, xyz.ctypes.data))
        out, k = [], 0
        for _, E, nu in self.blocks():
            out.append(xyz[k:k + E * nu].reshape(E, nu, 3))
            k += E * nu
        return out

    def split(self, flat):
        """Split a flat state (numpy or torch) into per-type (E, 5, N_u) views."""
        out, k = [], 0
        for _, E, nu in self.blocks():
            out.append(flat[k:k + E * 5 * nu].reshape(E, 5, nu))
            k += E * 5 * nu
        return out

    def connectivity(self):
        cnt = ctypes.c_int64()
        _check(self.ctx, self.lib.fr_connectivity(self.ctx, None, None, ctypes.byref(cnt)))
        nbr = np.empty(cnt.value, dtype=np.int64)
        isl = np.empty(cnt.value, dtype=np.int8)
        _check(self.ctx, self.lib.fr_connectivity(self.ctx, nbr.ctypes.data, isl.ctypes.data, ctypes.byref(cnt)))
        return nbr, isl

    # ---- device calls (torch tensors, float64, contiguous, on the GPU) ----
    @staticmethod
    def _dev(t, n):
        if t.dtype.itemsize != 8 or not t.is_contiguous() or t.numel() != n or t.device.type != "cuda":
            raise FrError("expected a contiguous float64 device tensor of %d elements" % n)
        return ctypes.c_void_p(t.data_ptr())

    def rhs(self, u, du):
        _check(self.ctx, self.lib.fr_rhs(self.ctx, self._dev(u, self.n_state), self._dev(du, self.n_state)))

    def rhs_noalloc(self, u, du):
        """du = R(u) with the work buffers in the library's static device
        scratch (no allocation); the mesh must be on the device already."""
        _check(self.ctx, self.lib.fr_rhs_noalloc(self.ctx, self._dev(u, self.n_state), self._dev(du, self.n_state)))

    def rhs_stages(self, u, du, mask):
        _check(self.ctx, self.lib.fr_rhs_stages(self.ctx, self._dev(u, self.n_state), self._dev(du, self.n_state),
                                                int(mask)))

    def set_state(self, u):
        if isinstance(u, np.ndarray):
            u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
            if u.size != self.n_state:
                raise FrError("state size mismatch")
            _check(self.ctx, self.lib.fr_set_state(self.ctx, u.ctypes.data, 0))
        else:
            _check(self.ctx, self.lib.fr_set_state(self.ctx, self._dev(u, self.n_state), 1))

    def get_state(self, out=None):
        if out is None:
            out = np.empty(self.n_state)
            _check(self.ctx, self.lib.fr_get_state(self.ctx, out.ctypes.data, 0))
            return out
        _check(self.ctx, self.lib.fr_get_state(self.ctx, self._dev(out, self.n_state), 1))
        return out

    def rk4(self, dt, nsteps=1):
        _check(self.ctx, self.lib.fr_rk4_step(self.ctx, float(dt), int(nsteps)))

    def integrals(self):
        out = np.empty(5)
        _check(self.ctx, self.lib.fr_integrals(self.ctx, out.ctypes.data))
        return out


class Pool:
    """Serving pool (fr_pool_*): continuous batching of independent solves.

    submit() queues a periodic-box request; step() runs one scheduling round
    (one RK4 step of every admitted request in shared launches, admissions by
    device footprint, retirement).  Host buffers given as u_init / u_out are
    kept referenced here until the request is done.
    """

    QUEUED, ACTIVE, DONE, FAILED = 0, 1, 2, 3

    def __init__(self, budget_bytes, max_active=64, prec="fp32", stream=None, **phys):
        self.lib = load_library()
        ph = physics(prec=prec, form="fused", **phys)
        c = ctypes.c_void_p()
        st = None if stream is None else ctypes.c_void_p(stream)
        _check(None, self.lib.fr_pool_create(ctypes.byref(ph), st, int(budget_bytes), int(max_active),
                                             ctypes.byref(c)))
        self.pool = c
        self._keep = {}

    def __del__(self):
        if getattr(self, "pool", None):
            self.lib.fr_pool_destroy(self.pool)
            self.pool = None

    @staticmethod
    def request(n, p, kind="hex", nsteps=1, dt=1e-4, lo=-np.pi, hi=np.pi, u_init=None, tgv_p0=0.0, u_out=None):
        nx, ny, nz = (n, n, n) if np.isscalar(n) else n
        return FrRequest(nx, ny, nz, lo, hi, p, MESH_KIND[kind], dt, nsteps,
                         None if u_init is None else u_init.ctypes.data, tgv_p0,
                         None if u_out is None else u_out.ctypes.data)

    def footprint(self, **req):
        r = self.request(**req)
        b, ns = ctypes.c_int64(), ctypes.c_int64()
        _check(self.pool, self.lib.fr_pool_footprint(self.pool, ctypes.byref(r), ctypes.byref(b), ctypes.byref(ns)),
               pool=True)
        return b.value, ns.value

    def submit(self, **req):
        """Queue a request; returns its id.  u_init / u_out: float64 numpy
        arrays of n_state entries (library layout) or None."""
        for k in ("u_init", "u_out"):
            a = req.get(k)
            if a is not None and (not isinstance(a, np.ndarray) or a.dtype != np.float64 or
                                  not a.flags.c_contiguous):
                raise FrError(k + " must be a contiguous float64 numpy array")
        if req.get("u_init") is not None or req.get("u_out") is not None:
            _, ns = self.footprint(**req)
            for k in ("u_init", "u_out"):
                if req.get(k) is not None and req[k].size != ns:
                    raise FrError("%s must hold %d doubles" % (k, ns))
        r = self.request(**req)
        i = ctypes.c_int64()
        _check(self.pool, self.lib.fr_pool_submit(self.pool, ctypes.byref(r), ctypes.byref(i)), pool=True)
        self._keep[i.value] = (req.get("u_init"), req.get("u_out"))
        return i.value

    def step(self):
        """One scheduling round; returns (stats dict, admitted ids, finished ids)."""
        s = FrPoolStats()
        _check(self.pool, self.lib.fr_pool_step(self.pool, ctypes.byref(s)), pool=True)
        na, nf = ctypes.c_int(), ctypes.c_int()
        cap = max(s.n_admitted, s.n_finished, 1)
        adm = np.empty(cap, dtype=np.int64)
        fin = np.empty(cap, dtype=np.int64)
        _check(self.pool, self.lib.fr_pool_events(self.pool, adm.ctypes.data, ctypes.byref(na), fin.ctypes.data,
                                                  ctypes.byref(nf), cap), pool=True)
        for i in fin[:nf.value]:
            self._keep.pop(int(i), None)
        stats = {k: getattr(s, k) for k, _ in FrPoolStats._fields_}
        return stats, adm[:na.value].tolist(), fin[:nf.value].tolist()

    def inject_prepare_error(self, rid):
        """Testing aid: make the host set-up of queued request rid fail."""
        _check(self.pool, self.lib.fr_pool_inject_prepare_error(self.pool, int(rid)), pool=True)

    def last_error(self):
        return self.lib.fr_pool_last_error(self.pool).decode()

    def query(self, rid):
        st, sd = ctypes.c_int(), ctypes.c_int()
        _check(self.pool, self.lib.fr_pool_query(self.pool, int(rid), ctypes.byref(st), ctypes.byref(sd)), pool=True)
        return st.value, sd.value
