"""Python binding of libmsl (the C-ABI in include/msl.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory (the workspace and the caller's
input / output tensors) and the HIP stream.  The library is loaded from the
package directory; a missing build is an error (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsl.so")

MSL_OK, MSL_EINVAL, MSL_ENOMEM, MSL_EHIP, MSL_EUNSTABLE, MSL_ESTATE = 0, -1, -2, -3, -4, -5
_ERRNAMES = {-1: "MSL_EINVAL", -2: "MSL_ENOMEM", -3: "MSL_EHIP", -4: "MSL_EUNSTABLE",
             -5: "MSL_ESTATE"}


class MslError(RuntimeError):
    def __init__(self, code, what, detail=""):
        self.code = code
        super().__init__(f"{what}: {_ERRNAMES.get(code, code)} {detail}".strip())


class MslConfig(C.Structure):
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
        ("check_every", C.c_int), ("mlp_hidden", C.c_int), ("mlp_check_every", C.c_int),
        ("u_ref", C.c_double * 3), ("T_ref", C.c_double), ("store_u", C.c_double * 3),
        ("tau2", C.c_double), ("pond", C.c_int), ("crit_margin", C.c_int),
    ]

# fields a workload may leave out: the lattice frame, the plain storage scale, BGK
_DEFAULTS = {"u_ref": (0.0, 0.0, 0.0), "T_ref": 1.0, "store_u": (0.0, 0.0, 0.0), "tau2": 0.0, "pond": 0,
             "crit_margin": 0}


_lib = None

# exported symbols of include/msl.h
SYMBOLS = [
    "msl_workspace_bytes", "msl_create", "msl_destroy", "msl_last_error", "msl_get_dt",
    "msl_init", "msl_set_mask", "msl_get_mask", "msl_step", "msl_get_step", "msl_macros",
    "msl_get_populations", "msl_set_populations", "msl_conservation", "msl_get_state",
    "msl_set_state", "msl_mlp_dims", "msl_collect_snapshots", "msl_mlp_set_weights",
    "msl_mlp_get_weights", "msl_mlp_train", "msl_mlp_grad", "msl_mlp_forward",
    "msl_mlp_get_flags", "msl_mlp_set_flags", "msl_num_check_tiles", "msl_profile",
    "msl_profile_read", "msl_device_copy", "msl_mlp_grad_noalloc", "msl_error_norms",
    "msl_pond_frames", "msl_pond_iterations", "msl_set_graph",
]


def lib():
    """The loaded libmsl.so (raises if the HIP build is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libmsl.so not built at {LIB_PATH}; run python paper_2102_12559_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, sz = C.c_void_p, C.c_size_t
        L.msl_workspace_bytes.argtypes = [C.POINTER(MslConfig), C.POINTER(sz)]
        L.msl_create.argtypes = [C.POINTER(MslConfig), vp, sz, vp, C.POINTER(vp)]
        L.msl_destroy.argtypes = [vp]
        L.msl_destroy.restype = None
        L.msl_last_error.argtypes = [vp]
        L.msl_last_error.restype = C.c_char_p
        L.msl_get_dt.argtypes = [vp, C.POINTER(C.c_double)]
        L.msl_init.argtypes = [vp, vp, vp, vp]
        L.msl_set_mask.argtypes = [vp, vp]
        L.msl_get_mask.argtypes = [vp, vp]
        L.msl_step.argtypes = [vp, C.c_int]
        L.msl_set_graph.argtypes = [vp, C.c_int]
        L.msl_get_step.argtypes = [vp, C.POINTER(C.c_long)]
        L.msl_macros.argtypes = [vp, vp, vp, vp]
        L.msl_get_populations.argtypes = [vp, C.c_int, C.c_int, vp]
        L.msl_set_populations.argtypes = [vp, C.c_int, C.c_int, vp]
        L.msl_conservation.argtypes = [vp, C.POINTER(C.c_double)]
        L.msl_error_norms.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_double)]
        L.msl_pond_frames.argtypes = [vp, vp]
        L.msl_pond_iterations.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.msl_get_state.argtypes = [vp, vp, C.POINTER(sz)]
        L.msl_set_state.argtypes = [vp, vp, sz]
        L.msl_mlp_dims.argtypes = [vp] + [C.POINTER(C.c_int)] * 4
        L.msl_collect_snapshots.argtypes = [vp, vp, vp, C.c_int, C.POINTER(C.c_int)]
        L.msl_mlp_set_weights.argtypes = [vp, vp, vp, vp, vp, vp]
        L.msl_mlp_get_weights.argtypes = [vp, vp]
        L.msl_mlp_train.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_float, vp]
        L.msl_mlp_grad.argtypes = [vp, vp, vp, C.c_int, C.POINTER(C.c_float), vp]
        L.msl_mlp_grad_noalloc.argtypes = [vp, vp, vp, C.c_int, C.POINTER(C.c_float), vp]
        L.msl_mlp_forward.argtypes = [vp, vp, C.c_int, vp]
        L.msl_mlp_get_flags.argtypes = [vp, vp]
        L.msl_mlp_set_flags.argtypes = [vp, vp]
        L.msl_num_check_tiles.argtypes = [vp, C.POINTER(C.c_int)]
        L.msl_profile.argtypes = [vp, C.c_int]
        L.msl_profile_read.argtypes = [vp, C.POINTER(C.c_double)]
        L.msl_device_copy.argtypes = [vp, vp, sz, vp]
        _lib = L
    return _lib


def make_config(cfg: dict) -> MslConfig:
    c = MslConfig()
    for name, _ in MslConfig._fields_:
        v = cfg.get(name, _DEFAULTS.get(name, 0))
        if name == "bc":
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
                c.slot_edge[k] = float(v[k]) if v else 0.0
        elif name in ("u_ref", "store_u"):
            arr = getattr(c, name)
            for k in range(3):
                arr[k] = float(v[k]) if k < len(v) else 0.0
        else:
            setattr(c, name, v)
    return c


def workspace_bytes(cfg: dict) -> int:
    c = make_config(cfg)
    n = C.c_size_t()
    rc = lib().msl_workspace_bytes(C.byref(c), C.byref(n))
    if rc:
        raise MslError(rc, "msl_workspace_bytes")
    return n.value


def device_copy(dst, src, stream):
    """Plain device copy (bandwidth reference); torch tensors of equal byte size."""
    nbytes = src.numel() * src.element_size()
    rc = lib().msl_device_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes,
                               C.c_void_p(stream.cuda_stream))
    if rc:
        raise MslError(rc, "msl_device_copy")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Solver:
    """One msl context: workspace and stream from PyTorch, state on the GPU."""

    def __init__(self, cfg: dict, device="cuda"):
        import torch
        self.torch = torch
        self.cfg = dict(cfg)
        self.dim = cfg["dim"]
        self.shape = (cfg["nz"] if cfg["dim"] == 3 else 1, cfg["ny"], cfg["nx"])
        self.ncell = int(np.prod(self.shape))
        self.Q = [cfg["n_low"] ** self.dim] + ([cfg["n_high"] ** self.dim] if cfg["n_high"] else [])
        self.device = torch.device(device)
        self._c = make_config(cfg)
        nbytes = workspace_bytes(cfg)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self._ctx = C.c_void_p()
        rc = lib().msl_create(C.byref(self._c), _ptr(self.ws), nbytes,
                              C.c_void_p(self.stream.cuda_stream), C.byref(self._ctx))
        if rc:
            raise MslError(rc, "msl_create")

    def close(self):
        if getattr(self, "_ctx", None):
            lib().msl_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc:
            raise MslError(rc, what, lib().msl_last_error(self._ctx).decode())

    # --- the C-ABI verbs -------------------------------------------------
    @property
    def dt(self):
        d = C.c_double()
        self._check(lib().msl_get_dt(self._ctx, C.byref(d)), "msl_get_dt")
        return d.value

    def _dev(self, a, dtype):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=dtype).contiguous()
        return t.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=self.device).contiguous()

    def set_mask(self, mask):
        m = self._dev(np.asarray(mask).reshape(-1) if not isinstance(mask, self.torch.Tensor)
                      else mask.reshape(-1), self.torch.uint8)
        self._check(lib().msl_set_mask(self._ctx, _ptr(m)), "msl_set_mask")

    def get_mask(self):
        m = self.torch.empty(self.ncell, dtype=self.torch.uint8, device=self.device)
        self._check(lib().msl_get_mask(self._ctx, _ptr(m)), "msl_get_mask")
        return m.reshape(self.shape)

    def init(self, rho, u, T=None):
        f64 = self.torch.float64
        r = self._dev(rho, f64).reshape(-1)
        uu = self._dev(u, f64).reshape(-1)
        TT = self._dev(T if T is not None else np.ones(self.ncell), f64).reshape(-1)
        self._check(lib().msl_init(self._ctx, _ptr(r), _ptr(uu), _ptr(TT)), "msl_init")
        self._keep = (r, uu, TT)

    def step(self, n=1):
        self._check(lib().msl_step(self._ctx, int(n)), "msl_step")

    def set_graph(self, mode):
        """0: launch by launch (default); 1: blocks of steps as HIP graphs; 2: as 1
        with the two sets' stream-collide launches on parallel graph branches."""
        self._check(lib().msl_set_graph(self._ctx, int(mode)), "msl_set_graph")

    @property
    def step_count(self):
        s = C.c_long()
        lib().msl_get_step(self._ctx, C.byref(s))
        return s.value

    def macros(self):
        t = self.torch
        rho = t.empty(self.ncell, dtype=t.float64, device=self.device)
        u = t.empty(self.dim * self.ncell, dtype=t.float64, device=self.device)
        T = t.empty(self.ncell, dtype=t.float64, device=self.device)
        self._check(lib().msl_macros(self._ctx, _ptr(rho), _ptr(u), _ptr(T)), "msl_macros")
        return rho.reshape(self.shape), u.reshape((self.dim,) + self.shape), T.reshape(self.shape)

    def get_populations(self, which, fg=0):
        t = self.torch
        out = t.empty((self.Q[which], self.ncell), dtype=t.float64, device=self.device)
        self._check(lib().msl_get_populations(self._ctx, which, fg, _ptr(out)),
                    "msl_get_populations")
        return out

    def set_populations(self, which, data, fg=0):
        d = self._dev(data, self.torch.float64).reshape(self.Q[which], self.ncell)
        self._check(lib().msl_set_populations(self._ctx, which, fg, _ptr(d)),
                    "msl_set_populations")
        self._keep_pops = d

    def conservation(self):
        out = (C.c_double * 5)()
        self._check(lib().msl_conservation(self._ctx, out), "msl_conservation")
        return np.array(out[:])

    def error_norms(self, rho_ref=None, u_ref=None, T_ref=None):
        """Relative L2 and max error norms of rho, u, T against reference
        fields (msl_error_norms); returns {"rho": (l2, max), "u": ..., "T": ...}."""
        t = self.torch
        refs = [None if r is None else self._dev(r, t.float64).contiguous().reshape(-1)
                for r in (rho_ref, u_ref, T_ref)]
        if refs[0] is not None and refs[0].numel() != self.ncell:
            raise ValueError("rho_ref: one value per cell")
        if refs[1] is not None and refs[1].numel() != self.dim * self.ncell:
            raise ValueError("u_ref: dim values per cell")
        if refs[2] is not None and refs[2].numel() != self.ncell:
            raise ValueError("T_ref: one value per cell")
        out = (C.c_double * 6)()
        self._check(lib().msl_error_norms(self._ctx, *[None if r is None else _ptr(r) for r in refs], out),
                    "msl_error_norms")
        return {"rho": (out[0], out[1]), "u": (out[2], out[3]), "T": (out[4], out[5])}

    def pond_frames(self):
        """co-moving frames: each cell's frame (u_x, u_y, u_z, T) as [4][cells]"""
        out = self.torch.empty((4, self.ncell), dtype=self.torch.float64, device=self.device)
        self._check(lib().msl_pond_frames(self._ctx, _ptr(out)), "msl_pond_frames")
        return out

    def pond_iterations(self):
        m, mx = C.c_double(), C.c_int()
        self._check(lib().msl_pond_iterations(self._ctx, C.byref(m), C.byref(mx)), "msl_pond_iterations")
        return m.value, mx.value

    def get_state(self) -> bytes:
        n = C.c_size_t()
        self._check(lib().msl_get_state(self._ctx, None, C.byref(n)), "msl_get_state")
        buf = C.create_string_buffer(n.value)
        self._check(lib().msl_get_state(self._ctx, buf, C.byref(n)), "msl_get_state")
        return buf.raw[: n.value]

    def set_state(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        self._check(lib().msl_set_state(self._ctx, buf, len(data)), "msl_set_state")

    # --- measurement --------------------------------------------------------
    PROFILE_CLASSES = ("ghost_fill", "stream_collide_low", "stream_collide_high",
                       "band_convert", "criterion_switch", "closure")

    def profile(self, enable=True, every=1):
        """Time the launches of every `every`-th step (HIP events)."""
        self._check(lib().msl_profile(self._ctx, int(every) if enable else 0), "msl_profile")

    def profile_read(self):
        st = (C.c_double * 24)()
        self._check(lib().msl_profile_read(self._ctx, st), "msl_profile_read")
        a = np.array(st[:]).reshape(6, 4)
        return {k: dict(launches=a[i, 0], ms=a[i, 1], bytes=a[i, 2], cells=a[i, 3])
                for i, k in enumerate(self.PROFILE_CLASSES)}

    # --- learned closure --------------------------------------------------
    def mlp_dims(self):
        v = [C.c_int() for _ in range(4)]
        self._check(lib().msl_mlp_dims(self._ctx, *[C.byref(x) for x in v]), "msl_mlp_dims")
        return tuple(x.value for x in v)  # F, O, H, P

    def collect_snapshots(self, max_rows):
        t = self.torch
        F, O, _, _ = self.mlp_dims()
        X = t.empty((max_rows, F), dtype=t.float32, device=self.device)
        Y = t.empty((max_rows, O), dtype=t.float32, device=self.device)
        n = C.c_int()
        self._check(lib().msl_collect_snapshots(self._ctx, _ptr(X), _ptr(Y), int(max_rows),
                                                C.byref(n)), "msl_collect_snapshots")
        return X[: n.value], Y[: n.value]

    def mlp_set_weights(self, params, xmean, xstd, tmean, tstd):
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (params, xmean, xstd, tmean, tstd)]
        self._check(lib().msl_mlp_set_weights(self._ctx, *[a.ctypes.data_as(C.c_void_p) for a in arrs]),
                    "msl_mlp_set_weights")

    def mlp_get_weights(self):
        P = self.mlp_dims()[3]
        out = np.zeros(P, dtype=np.float32)
        self._check(lib().msl_mlp_get_weights(self._ctx, out.ctypes.data_as(C.c_void_p)),
                    "msl_mlp_get_weights")
        return out

    def mlp_train(self, X, Y, batch=1024, epochs=1, lr=1e-3):
        t = self.torch
        X = X.to(self.device, t.float32).contiguous()
        Y = Y.to(self.device, t.float32).contiguous()
        n = X.shape[0]
        steps = epochs * ((n + batch - 1) // batch)
        log = np.zeros(steps, dtype=np.float32)
        self._check(lib().msl_mlp_train(self._ctx, _ptr(X), _ptr(Y), n, batch, epochs,
                                        C.c_float(lr), log.ctypes.data_as(C.c_void_p)),
                    "msl_mlp_train")
        return log

    def mlp_grad(self, X, Y):
        t = self.torch
        X = X.to(self.device, t.float32).contiguous()
        Y = Y.to(self.device, t.float32).contiguous()
        P = self.mlp_dims()[3]
        g = t.empty(P, dtype=t.float32, device=self.device)
        loss = C.c_float()
        self._check(lib().msl_mlp_grad(self._ctx, _ptr(X), _ptr(Y), X.shape[0], C.byref(loss), _ptr(g)),
                    "msl_mlp_grad")
        return loss.value, g

    def mlp_grad_noalloc(self, X, Y):
        """msl_mlp_grad with its partials in the library's static scratch array."""
        t = self.torch
        X = X.to(self.device, t.float32).contiguous()
        Y = Y.to(self.device, t.float32).contiguous()
        P = self.mlp_dims()[3]
        g = t.empty(P, dtype=t.float32, device=self.device)
        loss = C.c_float()
        self._check(lib().msl_mlp_grad_noalloc(self._ctx, _ptr(X), _ptr(Y), X.shape[0], C.byref(loss),
                                               _ptr(g)), "msl_mlp_grad_noalloc")
        return loss.value, g

    def mlp_forward(self, X):
        t = self.torch
        X = X.to(self.device, t.float32).contiguous()
        O = self.mlp_dims()[1]
        Y = t.empty((X.shape[0], O), dtype=t.float32, device=self.device)
        self._check(lib().msl_mlp_forward(self._ctx, _ptr(X), X.shape[0], _ptr(Y)), "msl_mlp_forward")
        return Y

    def num_check_tiles(self):
        n = C.c_int()
        self._check(lib().msl_num_check_tiles(self._ctx, C.byref(n)), "msl_num_check_tiles")
        return n.value

    def mlp_get_flags(self):
        f = self.torch.empty(self.num_check_tiles(), dtype=self.torch.uint8, device=self.device)
        self._check(lib().msl_mlp_get_flags(self._ctx, _ptr(f)), "msl_mlp_get_flags")
        return f

    def mlp_set_flags(self, flags):
        f = self._dev(flags, self.torch.uint8)
        self._check(lib().msl_mlp_set_flags(self._ctx, _ptr(f)), "msl_mlp_set_flags")
