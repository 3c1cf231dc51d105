"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU leg of the benchmark import
this module; the product path never does.
"""
from __future__ import annotations

import ctypes as C
import os

import math

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None


class OrConfig(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("n_low", C.c_int), ("n_high", C.c_int), ("thermal", C.c_int),
        ("tau", C.c_double), ("cv", C.c_double), ("cfl", C.c_double),
        ("tau_mode", C.c_int), ("mu_exp", C.c_double), ("tau_ref_rho", C.c_double),
        ("tau_ref_T", C.c_double), ("rho0", C.c_double), ("T0", C.c_double),
        ("store", C.c_int), ("lift_mode", C.c_int),
        ("bc", C.c_int * 6), ("bc_state", (C.c_double * 5) * 6),
        ("slot_state", (C.c_double * 5) * 6), ("slot", (C.c_int * 4) * 6),
        ("slot_edge", C.c_double * 6),
        ("crit_kind", C.c_int), ("crit_thr", C.c_double), ("crit_every", C.c_int),
        ("u_ref", C.c_double * 3), ("T_ref", C.c_double), ("store_u", C.c_double * 3),
        ("tau2", C.c_double), ("crit_margin", C.c_int),
    ]

# fields of the run configuration that default when a workload leaves them out
_DEFAULTS = {"u_ref": (0.0, 0.0, 0.0), "T_ref": 1.0, "store_u": (0.0, 0.0, 0.0), "tau2": 0.0,
             "crit_margin": 0}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from oracle import build as _b
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        _lib.or_dt.restype = C.c_double
        _lib.or_round_fp16.restype = C.c_double
        _lib.or_round_fp16.argtypes = [C.c_double]
        _lib.or_round_bf16.restype = C.c_double
        _lib.or_round_bf16.argtypes = [C.c_double]
        _lib.or_lagrange3.argtypes = [C.c_double, dp]
        _lib.or_lattice_feq.argtypes = [C.c_int, C.c_int, C.c_double, dp, C.c_double, dp]
        _lib.or_lift.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int,
                                 dp, dp, dp, dp]
        _lib.or_project.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp, dp]
        _lib.or_step_count.restype = C.c_long
        _lib.or_pond_dt.restype = C.c_double
        _lib.or_pond_dt.argtypes = [C.c_void_p]
        _lib.or_pond_transfer.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp]
        _lib.or_set_threads.argtypes = [C.c_int]
        _lib.or_set_threads.restype = C.c_int
        _lib.or_adam.argtypes = [dp, dp, dp, dp, C.c_int, C.c_int, C.c_double, C.c_double,
                                 C.c_double, C.c_double]
        _lib.or_mlp_features.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, dp, dp, dp]
        _lib.or_mlp_targets.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, dp,
                                        dp, dp]
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with {rc}")


def make_config(cfg: dict) -> OrConfig:
    c = OrConfig()
    for name, _ in OrConfig._fields_:
        v = cfg.get(name, _DEFAULTS.get(name)) if name in _DEFAULTS else cfg[name]
        if name in ("bc",):
            for k in range(6):
                c.bc[k] = int(v[k])
        elif name in ("bc_state", "slot_state"):
            arr = getattr(c, name)
            for k in range(6):
                for m in range(5):
                    arr[k][m] = float(v[k][m])
        elif name == "slot":
            for k in range(6):
                for m in range(4):
                    c.slot[k][m] = int(v[k][m])
        elif name == "slot_edge":
            for k in range(6):
                c.slot_edge[k] = float(v[k])
        elif name in ("u_ref", "store_u"):
            arr = getattr(c, name)
            for k in range(3):
                arr[k] = float(v[k]) if k < len(v) else 0.0
        else:
            setattr(c, name, v)
    return c


# ---------------------------------------------------------------------------
# lattice-level helpers
# ---------------------------------------------------------------------------

def set_threads(n):
    """OpenMP threads of the oracle's stepper; returns the previous count."""
    return lib().or_set_threads(int(n))


def gh_rule(n):
    x = np.zeros(n)
    w = np.zeros(n)
    _check(lib().or_gh_rule(n, _p(x), _p(w)), "gh_rule")
    return x, w


def lattice_feq(dim, n, rho, u, theta):
    out = np.zeros(n ** dim)
    uu = np.zeros(3)
    uu[:dim] = u[:dim]
    _check(lib().or_lattice_feq(dim, n, float(rho), _p(uu), float(theta), _p(out)), "feq")
    return out


def moment_matrix(dim, n):
    Q = n ** dim
    M = np.zeros((Q, Q))
    Mi = np.zeros((Q, Q))
    _check(lib().or_moment_matrix(dim, n, _p(M), _p(Mi)), "moment_matrix")
    return M, Mi


def lift(dim, nq, nQ, fq, gq=None, thermal=0, cv=1.5, mode=0):
    fq = np.ascontiguousarray(fq, dtype=np.float64)
    fQ = np.zeros(nQ ** dim)
    gQ = np.zeros(nQ ** dim) if gq is not None else None
    gqa = np.ascontiguousarray(gq, dtype=np.float64) if gq is not None else None
    _check(lib().or_lift(dim, nq, nQ, thermal, cv, mode, _p(fq), _p(gqa), _p(fQ), _p(gQ)), "lift")
    return (fQ, gQ) if gq is not None else fQ


def project(dim, nQ, nq, fQ, gQ=None):
    fQ = np.ascontiguousarray(fQ, dtype=np.float64)
    fq = np.zeros(nq ** dim)
    gq = np.zeros(nq ** dim) if gQ is not None else None
    gQa = np.ascontiguousarray(gQ, dtype=np.float64) if gQ is not None else None
    _check(lib().or_project(dim, nQ, nq, _p(fQ), _p(gQa), _p(fq), _p(gq)), "project")
    return (fq, gq) if gQ is not None else fq


def lagrange3(xi):
    a = np.zeros(3)
    lib().or_lagrange3(float(xi), _p(a))
    return a


def round_fp16(v):
    return lib().or_round_fp16(float(v))


def round_bf16(v):
    return lib().or_round_bf16(float(v))


def mlp_nparams(F, H, O):
    return lib().or_mlp_nparams(F, H, O)


def mlp_dims(dim, nq, nQ):
    F = C.c_int()
    O = C.c_int()
    lib().or_mlp_dims(dim, nq, nQ, C.byref(F), C.byref(O))
    return F.value, O.value


def mlp_forward(params, F, H, O, X, bf16=False):
    X = np.ascontiguousarray(X, dtype=np.float64)
    n = X.shape[0]
    Y = np.zeros((n, O))
    p = np.ascontiguousarray(params, dtype=np.float64)
    _check(lib().or_mlp_forward(_p(p), F, H, O, n, _p(X), _p(Y), int(bf16)), "mlp_forward")
    return Y


def mlp_loss_grad(params, F, H, O, X, T):
    X = np.ascontiguousarray(X, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    p = np.ascontiguousarray(params, dtype=np.float64)
    g = np.zeros_like(p)
    loss = C.c_double()
    _check(lib().or_mlp_loss_grad(_p(p), F, H, O, X.shape[0], _p(X), _p(T), C.byref(loss), _p(g)),
           "mlp_loss_grad")
    return loss.value, g


def adam(p, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    lib().or_adam(_p(p), _p(m), _p(v), _p(np.ascontiguousarray(g)), p.size, t, lr, b1, b2, eps)


def mlp_features(dim, nq, fq, gq=None, thermal=0, cv=1.5):
    F, _ = mlp_dims(dim, nq, nq + 1)
    out = np.zeros(F)
    fq = np.ascontiguousarray(fq, dtype=np.float64)
    gqa = np.ascontiguousarray(gq, dtype=np.float64) if gq is not None else None
    _check(lib().or_mlp_features(dim, nq, thermal, cv, _p(fq), _p(gqa), _p(out)), "features")
    return out


def mlp_targets(dim, nq, nQ, fQ, gQ=None, thermal=0, cv=1.5):
    _, O = mlp_dims(dim, nq, nQ)
    out = np.zeros(O)
    fQ = np.ascontiguousarray(fQ, dtype=np.float64)
    gQa = np.ascontiguousarray(gQ, dtype=np.float64) if gQ is not None else None
    _check(lib().or_mlp_targets(dim, nq, nQ, thermal, cv, _p(fQ), _p(gQa), _p(out)), "targets")
    return out


# ---------------------------------------------------------------------------
# stepper
# ---------------------------------------------------------------------------

class Oracle:
    """The multi-scale step on host FP64 arrays (same verbs as the GPU library)."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self._c = make_config(cfg)
        self._ctx = C.c_void_p()
        _check(lib().or_create(C.byref(self._c), C.byref(self._ctx)), "create")
        self.dim = cfg["dim"]
        self.shape = (cfg["nz"] if cfg["dim"] == 3 else 1, cfg["ny"], cfg["nx"])
        self.ncell = int(np.prod(self.shape))
        self.Q = [cfg["n_low"] ** self.dim] + ([cfg["n_high"] ** self.dim] if cfg["n_high"] else [])

    def __del__(self):
        if getattr(self, "_ctx", None):
            lib().or_destroy(self._ctx)
            self._ctx = None

    @property
    def dt(self):
        return lib().or_dt(self._ctx)

    @property
    def reach(self):
        return lib().or_reach(self._ctx)

    def stencil(self, which):
        Q = self.Q[which]
        n0 = np.zeros((Q, self.dim), dtype=np.int32)
        a = np.zeros((Q, self.dim, 3))
        _check(lib().or_stencil(self._ctx, which, n0.ctypes.data_as(C.POINTER(C.c_int)), _p(a)),
               "stencil")
        return n0, a

    def set_mask(self, mask, convert=True):
        m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        fn = lib().or_set_mask if convert else lib().or_set_mask_raw
        _check(fn(self._ctx, m.ctypes.data_as(C.c_void_p)), "set_mask")

    def get_mask(self):
        m = np.zeros(self.ncell, dtype=np.uint8)
        lib().or_get_mask(self._ctx, m.ctypes.data_as(C.c_void_p))
        return m.reshape(self.shape)

    def eval_criterion(self):
        m = np.zeros(self.ncell, dtype=np.uint8)
        v = np.zeros(self.ncell)
        lib().or_eval_criterion(self._ctx, m.ctypes.data_as(C.c_void_p), _p(v))
        return m.reshape(self.shape), v.reshape(self.shape)

    def init(self, rho, u, T=None):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        T = np.ones(self.ncell) if T is None else np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
        _check(lib().or_init(self._ctx, _p(rho), _p(u), _p(T)), "init")

    def step(self, n=1):
        _check(lib().or_step(self._ctx, int(n)), "step")

    @property
    def step_count(self):
        return lib().or_step_count(self._ctx)

    def get_pops(self, which, fg=0):
        out = np.zeros((self.Q[which], self.ncell))
        _check(lib().or_get_pops(self._ctx, which, fg, _p(out)), "get_pops")
        return out

    def set_pops(self, which, data, fg=0):
        d = np.ascontiguousarray(data, dtype=np.float64).reshape(self.Q[which], self.ncell)
        _check(lib().or_set_pops(self._ctx, which, fg, _p(d)), "set_pops")

    def qeq(self, which, f, g=None):
        """Quasi-equilibria f*, g* of one cell's populations of lattice `which`."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        ga = np.ascontiguousarray(g, dtype=np.float64) if g is not None else np.zeros_like(f)
        fs = np.zeros_like(f)
        gs = np.zeros_like(f)
        _check(lib().or_qeq(self._ctx, which, _p(f), _p(ga), _p(fs), _p(gs)), "qeq")
        return fs, gs

    def macros(self):
        rho = np.zeros(self.ncell)
        u = np.zeros((self.dim, self.ncell))
        T = np.zeros(self.ncell)
        _check(lib().or_macros(self._ctx, _p(rho), _p(u), _p(T)), "macros")
        return rho.reshape(self.shape), u.reshape((self.dim,) + self.shape), T.reshape(self.shape)

    def conservation(self):
        out = np.zeros(5)
        lib().or_conservation(self._ctx, _p(out))
        return out

    def step_cells(self, cells):
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        Qm = self.Q[-1]
        f = np.zeros((cells.size, Qm))
        g = np.zeros((cells.size, Qm))
        _check(lib().or_step_cells(self._ctx, cells.size, cells.ctypes.data_as(C.c_void_p),
                                   _p(f), _p(g)), "step_cells")
        return f, g

    # learned closure
    def set_mlp(self, H, params, xmean, xstd, tmean, tstd, bf16=False, manual_check=False):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (params, xmean, xstd, tmean, tstd)]
        flags = (1 if bf16 else 0) | (2 if manual_check else 0)
        _check(lib().or_set_mlp(self._ctx, H, *[_p(a) for a in arrs], flags), "set_mlp")

    def ntiles(self):
        return int(np.prod([(s + 63) // 64 for s in self.shape]))

    def set_mlp_flags(self, flags):
        f = np.ascontiguousarray(flags, dtype=np.uint8)
        lib().or_set_mlp_flags(self._ctx, f.ctypes.data_as(C.c_void_p))

    def mlp_flags(self):
        n = self.ntiles()
        f = np.zeros(n, dtype=np.uint8)
        e1 = np.zeros(n)
        e2 = np.zeros(n)
        lib().or_get_mlp_flags(self._ctx, f.ctypes.data_as(C.c_void_p), _p(e1), _p(e2))
        return f, e1, e2

    def mlp_check(self):
        _check(lib().or_mlp_check(self._ctx), "mlp_check")

    def lift_cell(self, fq, gq=None, tile=0):
        fq = np.ascontiguousarray(fq, dtype=np.float64)
        gqa = np.ascontiguousarray(gq, dtype=np.float64) if gq is not None else np.zeros_like(fq)
        fQ = np.zeros(self.Q[1])
        gQ = np.zeros(self.Q[1])
        _check(lib().or_lift_cell(self._ctx, _p(fq), _p(gqa), int(tile), _p(fQ), _p(gQ)),
               "lift_cell")
        return (fQ, gQ) if gq is not None else fQ


def error_norms(rho, u, T, rho_ref=None, u_ref=None, T_ref=None):
    """Relative L2 and max error norms of macroscopic fields against reference
    fields, written out from their definition: for each field the square root
    of sum |x - x_ref|^2 over sum |x_ref|^2 (u: Euclidean norm over the
    components per cell; the root mean square of the difference where the
    reference is zero everywhere) and the largest |x - x_ref|.  Skipped
    fields give (0, 0)."""
    out = {}
    for name, x, r, vec in (("rho", rho, rho_ref, False), ("u", u, u_ref, True), ("T", T, T_ref, False)):
        if r is None:
            out[name] = (0.0, 0.0)
            continue
        x = np.asarray(x, dtype=np.float64)
        r = np.asarray(r, dtype=np.float64).reshape(x.shape)
        d = x - r
        if vec:
            dn = np.sqrt(np.sum(d.reshape(d.shape[0], -1) ** 2, axis=0))
            rn2 = np.sum(r ** 2)
        else:
            dn = np.abs(d).reshape(-1)
            rn2 = np.sum(r ** 2)
        sd = float(np.sum(dn ** 2))
        l2 = math.sqrt(sd / rn2) if rn2 > 0 else math.sqrt(sd / dn.size)
        out[name] = (l2, float(np.max(dn)))
    return out


class Pond:
    """The step in co-moving reference frames (PonD, Sec. II.C.1), one or two
    velocity sets, on host FP64 arrays."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self._c = make_config(cfg)
        self._ctx = C.c_void_p()
        _check(lib().or_pond_create(C.byref(self._c), C.byref(self._ctx)), "pond create")
        self.dim = cfg["dim"]
        self.shape = (cfg["nz"] if cfg["dim"] == 3 else 1, cfg["ny"], cfg["nx"])
        self.ncell = int(np.prod(self.shape))
        self.Q = cfg["n_low"] ** self.dim
        self.Qs = [cfg["n_low"] ** self.dim] + ([cfg["n_high"] ** self.dim] if cfg.get("n_high") else [])

    def __del__(self):
        if getattr(self, "_ctx", None):
            lib().or_pond_destroy(self._ctx)
            self._ctx = None

    @property
    def dt(self):
        return lib().or_pond_dt(self._ctx)

    def init(self, rho, u, T=None):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        T = np.ones(self.ncell) if T is None else np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
        _check(lib().or_pond_init(self._ctx, _p(rho), _p(u), _p(T)), "pond init")

    def step(self, n=1):
        _check(lib().or_pond_step(self._ctx, int(n)), "pond step")

    def macros(self):
        rho = np.zeros(self.ncell)
        u = np.zeros(self.dim * self.ncell)
        T = np.zeros(self.ncell)
        _check(lib().or_pond_macros(self._ctx, _p(rho), _p(u), _p(T)), "pond macros")
        return rho.reshape(self.shape), u.reshape((self.dim,) + self.shape), T.reshape(self.shape)

    def get_pops(self, which=0, fg=0):
        out = np.zeros((self.Qs[which], self.ncell))
        _check(lib().or_pond_get_pops(self._ctx, which, fg, _p(out)), "pond get_pops")
        return out

    def set_mask(self, mask, convert=True):
        m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        _check(lib().or_pond_set_mask(self._ctx, m.ctypes.data_as(C.c_void_p), int(convert)), "pond set_mask")

    def get_mask(self):
        out = np.zeros(self.ncell, dtype=np.uint8)
        _check(lib().or_pond_get_mask(self._ctx, out.ctypes.data_as(C.c_void_p)), "pond get_mask")
        return out.reshape(self.shape)

    def get_frames(self):
        out = np.zeros((4, self.ncell))
        _check(lib().or_pond_get_frames(self._ctx, _p(out)), "pond get_frames")
        return out

    def iterations(self):
        m = C.c_double()
        mx = C.c_int()
        lib().or_pond_iterations(self._ctx, C.byref(m), C.byref(mx))
        return m.value, mx.value


def dilate_mask(cfg, mask):
    """The criterion's margin applied to a 0/1 mask (or_dilate_mask)."""
    c = make_config(cfg)
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    out = np.zeros_like(m)
    _check(lib().or_dilate_mask(C.byref(c), m.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p)),
           "dilate_mask")
    return out.reshape(np.shape(mask))


def pond_transfer(dim, n, src, dst, f):
    """G_src^dst f (eq. fll) of one population vector; frames (u_x, u_y, u_z, T)"""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    s = np.ascontiguousarray(src, dtype=np.float64)
    d = np.ascontiguousarray(dst, dtype=np.float64)
    _check(lib().or_pond_transfer(dim, n, _p(s), _p(d), _p(f), _p(out)), "pond transfer")
    return out
