"""Python binding of libvlasov.so (include/vlasov.h): argument marshalling only.

Device memory comes from torch (the f pair and the workspace are uint8
tensors on the GPU) and the stream is torch's current stream; every step of
the solver runs in the library's HIP kernels.  There is no fallback: if the
library is not built, or no GPU is present, construction fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libvlasov.so")

OK, PENDING = 0, 1
E_INVAL, E_NOMEM, E_HIP, E_STATE, E_NOTFOUND, E_NONFINITE = -1, -2, -3, -4, -5, -6

K_DRIFT, K_DRIFT2, K_DENSITY, K_FORCE, K_KICK, K_MOMENTS, K_KICK_DRIFT2 = range(7)
KERNELS = ("drift", "drift2", "density", "force", "kick", "moments", "kick_drift2", "filter")


class VlasovError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"vlasov error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("model", C.c_int32), ("storage", C.c_int32), ("bc_x", C.c_int32), ("bc_p", C.c_int32),
                ("nx", C.c_int64), ("np", C.c_int64),
                ("xmin", C.c_double), ("xmax", C.c_double), ("pmin", C.c_double), ("pmax", C.c_double),
                ("dt", C.c_double), ("ring_eps", C.c_double), ("sheet_G", C.c_double),
                ("hist_cap", C.c_int64), ("spline", C.c_int32), ("splitting", C.c_int32),
                ("filter_every", C.c_int32), ("reserved", C.c_int32), ("filter_strength", C.c_double)]


class Moments(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("mass", "momentum", "kinetic", "potential", "energy", "mx", "my", "l2",
                                          "entropy", "neg_mass")]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class Tuning(C.Structure):
    _fields_ = [("drift_threads", C.c_int32), ("kick_rows", C.c_int32), ("kick_drift_width", C.c_int32),
                ("kick_drift_blocks", C.c_int32)]


IC_HOST, IC_WATERBAG, IC_WATERBAG_UM, IC_GAUSSIAN = 0, 1, 2, 3


class IC(C.Structure):
    """Initial condition generated on the device (vlasov_ic)."""
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("a0", C.c_double), ("a1", C.c_double),
                ("amp", C.c_double), ("seed", C.c_uint64)]


def ic_waterbag(x0: float, p0: float, amp: float = 0.0, seed: int = 0) -> IC:
    return IC(IC_WATERBAG, 0, float(x0), float(p0), float(amp), int(seed))


def ic_waterbag_um(U: float, M0: float, amp: float = 0.0, seed: int = 0) -> IC:
    return IC(IC_WATERBAG_UM, 0, float(U), float(M0), float(amp), int(seed))


def ic_gaussian(T: float, amp: float, seed: int = 0) -> IC:
    return IC(IC_GAUSSIAN, 0, float(T), 0.0, float(amp), int(seed))


class Request(C.Structure):
    _fields_ = [("p", Params), ("nsteps", C.c_int64), ("keep_f", C.c_int32), ("reserved", C.c_int32),
                ("ic", IC)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("reserved", C.c_int32), ("steps_done", C.c_int64),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double), ("m", Moments)]

    def as_dict(self) -> dict:
        d = {n: getattr(self, n) for n in ("status", "steps_done", "t_submit", "t_admit", "t_done")}
        d["moments"] = self.m.as_dict()
        return d


_D = C.POINTER(C.c_double)
_lib = None


def load() -> C.CDLL:
    """Load the in-tree HIP library (built by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        lib = C.CDLL(LIB_PATH)
        P = C.POINTER(Params)
        V = C.c_void_p
        sig = {
            "vlasov_f_bytes": (C.c_size_t, [P]),
            "vlasov_workspace_bytes": (C.c_size_t, [P]),
            "vlasov_init": (C.c_int, [P, _D, V, V, V, C.POINTER(V)]),
            "vlasov_init_static": (C.c_int, [P, _D, V, V, C.POINTER(V)]),
            "vlasov_set_external_force": (C.c_int, [V, _D]),
            "vlasov_step": (C.c_int, [V, C.c_int64]),
            "vlasov_set_graph": (C.c_int, [V, C.c_int32]),
            "vlasov_drift": (C.c_int, [V, C.c_int32]),
            "vlasov_force": (C.c_int, [V, _D, _D]),
            "vlasov_kick": (C.c_int, [V]),
            "vlasov_moments": (C.c_int, [V, C.POINTER(Moments)]),
            "vlasov_mag_history": (C.c_int, [V, _D, _D, C.c_int64, C.POINTER(C.c_int64)]),
            "vlasov_read_f": (C.c_int, [V, _D]),
            "vlasov_write_f": (C.c_int, [V, _D]),
            "vlasov_generate_ic": (C.c_int, [V, C.POINTER(IC)]),
            "vlasov_destroy": (C.c_int, [V]),
            "vlasov_last_error": (C.c_char_p, []),
            "vlasov_profile_enable": (C.c_int, [V, C.c_int32]),
            "vlasov_profile_read": (C.c_int, [V, C.c_int32, _D, C.POINTER(C.c_int64)]),
            "vlasov_kernel_name": (C.c_char_p, [C.c_int32]),
            "vlasov_device_copy": (C.c_int, [V, V, C.c_size_t, V]),
            "vlasov_tuning_candidates": (C.c_int, [C.POINTER(Tuning), C.c_int32, C.POINTER(C.c_int32)]),
            "vlasov_set_tuning": (C.c_int, [V, C.POINTER(Tuning)]),
            "vlasov_get_tuning": (C.c_int, [V, C.POINTER(Tuning)]),
            "vlasov_batch_scratch_bytes": (C.c_size_t, [C.c_int32]),
            "vlasov_batch_step": (C.c_int, [C.POINTER(V), C.c_int32, C.POINTER(C.c_int64), V, C.c_size_t,
                                            C.c_int32, C.c_int32]),
            "vlasov_request_footprint": (C.c_size_t, [P]),
            "vlasov_server_table_bytes": (C.c_size_t, [C.c_int32]),
            "vlasov_server_create": (C.c_int, [V, C.c_size_t, V, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                               C.POINTER(V)]),
            "vlasov_submit": (C.c_int, [V, C.POINTER(Request), _D, C.POINTER(C.c_uint64)]),
            "vlasov_poll": (C.c_int, [V, C.c_uint64, C.POINTER(Result), _D]),
            "vlasov_server_stats": (C.c_int, [V, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
            "vlasov_server_destroy": (C.c_int, [V]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(rc: int) -> int:
    if rc < 0:
        raise VlasovError(rc, load().vlasov_last_error().decode())
    return rc


def to_params(p, hist_cap: int = 0) -> Params:
    """From paper_1206_3229_amd.inputs.Params."""
    return Params(int(p.model), int(p.storage), int(p.bc_x), int(p.bc_p), int(p.nx), int(p.np_),
                  float(p.xmin), float(p.xmax), float(p.pmin), float(p.pmax), float(p.dt),
                  float(p.ring_eps), float(p.sheet_G), int(hist_cap), int(getattr(p, "spline", 0)),
                  int(getattr(p, "splitting", 0)), int(getattr(p, "filter_every", 0)), 0,
                  float(getattr(p, "filter_strength", 0.0)))


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the Vlasov solver runs only on the device")
    return torch


class Solver:
    """One simulation: f pair and workspace in device memory, steps on the current stream.

    static_workspace=True creates the context with vlasov_init_static: the
    workspace is the library's static device array (no workspace tensor), one
    such context per device at a time."""

    def __init__(self, params, f0: np.ndarray, hist_cap: int = 0, device: int | None = None,
                 static_workspace: bool = False):
        torch = _torch()
        lib = load()
        self.params = params
        self._p = to_params(params, hist_cap)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        fb = lib.vlasov_f_bytes(C.byref(self._p))
        wb = lib.vlasov_workspace_bytes(C.byref(self._p))
        if fb == 0 or wb == 0:
            raise VlasovError(E_INVAL, "invalid parameters")
        with torch.cuda.device(self.device):
            self.f_buf = torch.empty(fb, dtype=torch.uint8, device=self.device)
            self.ws_buf = None if static_workspace else torch.empty(wb, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        # f0: the initial f as an FP64 [np][nx] array, or an IC generated on the device
        gen = f0 if isinstance(f0, IC) else None
        if gen is None:
            f0 = np.ascontiguousarray(f0, dtype=np.float64)
            if f0.shape != (params.np_, params.nx):
                raise ValueError(f"f0 shape {f0.shape} != (np, nx) = {(params.np_, params.nx)}")
        f0p = None if gen is not None else _dptr(f0)
        ctx = C.c_void_p()
        if static_workspace:
            with torch.cuda.device(self.device):
                check(lib.vlasov_init_static(C.byref(self._p), f0p, C.c_void_p(self.f_buf.data_ptr()),
                                             C.c_void_p(self.stream.cuda_stream), C.byref(ctx)))
        else:
            check(lib.vlasov_init(C.byref(self._p), f0p, C.c_void_p(self.f_buf.data_ptr()),
                                  C.c_void_p(self.ws_buf.data_ptr()), C.c_void_p(self.stream.cuda_stream),
                                  C.byref(ctx)))
        self._ctx = ctx
        self.nx, self.np_ = params.nx, params.np_
        if gen is not None:
            self.generate_ic(gen)

    def generate_ic(self, ic: "IC"):
        """Replace f by an initial condition generated on the device."""
        check(load().vlasov_generate_ic(self._ctx, C.byref(ic)))

    # -- steps -----------------------------------------------------------
    def step(self, nsteps: int = 1):
        check(load().vlasov_step(self._ctx, int(nsteps)))

    def set_graph(self, steps_per_graph: int):
        """Steps per HIP graph launch in step() (0: no graphs)."""
        check(load().vlasov_set_graph(self._ctx, int(steps_per_graph)))

    def drift(self, npass: int = 1):
        check(load().vlasov_drift(self._ctx, int(npass)))

    def force(self):
        F = np.empty(self.nx)
        mm = np.zeros(2)
        check(load().vlasov_force(self._ctx, _dptr(F), _dptr(mm)))
        return F, (float(mm[0]), float(mm[1]))

    def kick(self):
        check(load().vlasov_kick(self._ctx))

    def set_external_force(self, F: np.ndarray):
        F = np.ascontiguousarray(F, dtype=np.float64)
        assert F.shape == (self.nx,)
        check(load().vlasov_set_external_force(self._ctx, _dptr(F)))

    # -- state -----------------------------------------------------------
    def read_f(self) -> np.ndarray:
        out = np.empty((self.np_, self.nx))
        check(load().vlasov_read_f(self._ctx, _dptr(out)))
        return out

    def write_f(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (self.np_, self.nx)
        check(load().vlasov_write_f(self._ctx, _dptr(f)))

    def moments(self) -> dict:
        m = Moments()
        check(load().vlasov_moments(self._ctx, C.byref(m)))
        return m.as_dict()

    def mag_history(self) -> np.ndarray:
        cap = self._p.hist_cap
        mx, my = np.zeros(max(cap, 1)), np.zeros(max(cap, 1))
        n = C.c_int64()
        check(load().vlasov_mag_history(self._ctx, _dptr(mx), _dptr(my), cap, C.byref(n)))
        k = min(n.value, cap)
        return np.stack([mx[:k], my[:k]], axis=1)

    # -- launch shapes ---------------------------------------------------
    def set_tuning(self, drift_threads: int, kick_rows: int, kick_drift_width: int = 0, kick_drift_blocks: int = 1):
        """kick_drift_width 0: separate kick and drift kernels; 230 or 486:
        the fused kernel on tiles of that width and kick_drift_blocks 16-row
        blocks (where the grid allows it)."""
        t = Tuning(int(drift_threads), int(kick_rows), int(kick_drift_width), int(kick_drift_blocks))
        check(load().vlasov_set_tuning(self._ctx, C.byref(t)))

    def get_tuning(self) -> tuple[int, int, int, int]:
        t = Tuning()
        check(load().vlasov_get_tuning(self._ctx, C.byref(t)))
        return t.drift_threads, t.kick_rows, t.kick_drift_width, t.kick_drift_blocks

    # -- measurement -----------------------------------------------------
    def profile(self, on: bool = True):
        check(load().vlasov_profile_enable(self._ctx, 1 if on else 0))

    def profile_read(self) -> dict:
        out = {}
        for k, name in enumerate(KERNELS):
            ms = C.c_double()
            n = C.c_int64()
            check(load().vlasov_profile_read(self._ctx, k, C.byref(ms), C.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def close(self):
        if getattr(self, "_ctx", None):
            load().vlasov_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


BATCH_GRAPH, BATCH_FUSE = 1, 2


def batch_step(solvers, nsteps, chunk_cycles: int = 16, use_graph: bool = True, fuse: bool = False):
    """Advance several solvers (one storage type, one stream) together with the
    batched persistent kernels; solver k by nsteps[k] steps.  fuse: the kick
    fused with the pair of half drifts after it, where a grid allows it."""
    torch = _torch()
    lib = load()
    n = len(solvers)
    nb = lib.vlasov_batch_scratch_bytes(int(chunk_cycles))
    if nb == 0:
        raise VlasovError(E_INVAL, "bad chunk_cycles")
    scratch = torch.empty(nb, dtype=torch.uint8, device=solvers[0].device)
    ctxs = (C.c_void_p * n)(*[s._ctx for s in solvers])
    steps = (C.c_int64 * n)(*[int(k) for k in nsteps])
    flags = (BATCH_GRAPH if use_graph else 0) | (BATCH_FUSE if fuse else 0)
    check(lib.vlasov_batch_step(ctxs, n, steps, C.c_void_p(scratch.data_ptr()), nb, int(chunk_cycles), flags))
    del scratch


class Server:
    """Continuous-batching request server over a torch-allocated device arena.

    The defaults are the shape measured fastest on the 512-request scan: up to
    128 requests per cycle, 64-cycle chunks replayed from HIP graphs, and the
    kick fused with the half drifts around it (BATCH_FUSE) for the requests
    that allow it."""

    def __init__(self, arena_bytes: int, storage: int = 1, max_slots: int = 128, chunk_cycles: int = 64,
                 use_graph: bool = True, device: int | None = None, fuse: bool = True):
        torch = _torch()
        lib = load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.storage = storage
        with torch.cuda.device(self.device):
            self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        srv = C.c_void_p()
        check(lib.vlasov_server_create(C.c_void_p(self.arena.data_ptr()), int(arena_bytes),
                                       C.c_void_p(self.stream.cuda_stream), int(storage), int(max_slots),
                                       int(chunk_cycles), (BATCH_GRAPH if use_graph else 0) | (BATCH_FUSE if fuse else 0),
                                       C.byref(srv)))
        self._srv = srv
        self._shapes = {}

    def submit(self, params, f0, nsteps: int, keep_f: bool = False) -> int:
        """f0: FP64 [np][nx] array, or an IC the server generates on the device."""
        if isinstance(f0, IC):
            req = Request(to_params(params, 0), int(nsteps), 1 if keep_f else 0, 0, f0)
            f0p = None
        else:
            f0 = np.ascontiguousarray(f0, dtype=np.float64)
            assert f0.shape == (params.np_, params.nx)
            req = Request(to_params(params, 0), int(nsteps), 1 if keep_f else 0, 0, IC())
            f0p = _dptr(f0)
        t = C.c_uint64()
        check(load().vlasov_submit(self._srv, C.byref(req), f0p, C.byref(t)))
        self._shapes[t.value] = (params.np_, params.nx, keep_f)
        return t.value

    def poll(self, ticket: int):
        """None while pending, else (result dict, f or None)."""
        np_, nx, keep = self._shapes.get(ticket, (1, 1, False))
        r = Result()
        f = np.empty((np_, nx)) if keep else None
        rc = check(load().vlasov_poll(self._srv, int(ticket), C.byref(r), _dptr(f) if f is not None else None))
        if rc == PENDING:
            return None
        self._shapes.pop(ticket, None)
        # a failed request returns no f
        return r.as_dict(), (f if r.status == OK else None)

    def stats(self):
        q, r, d = C.c_int64(), C.c_int64(), C.c_int64()
        check(load().vlasov_server_stats(self._srv, C.byref(q), C.byref(r), C.byref(d)))
        return q.value, r.value, d.value

    def close(self):
        if getattr(self, "_srv", None):
            load().vlasov_server_destroy(self._srv)
            self._srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tuning_candidates() -> list[tuple[int, int, int, int]]:
    """(drift_threads, kick_rows, kick_drift_width, kick_drift_blocks) of every compiled shape."""
    n = C.c_int32()
    check(load().vlasov_tuning_candidates(None, 0, C.byref(n)))
    arr = (Tuning * n.value)()
    check(load().vlasov_tuning_candidates(arr, n.value, C.byref(n)))
    return [(t.drift_threads, t.kick_rows, t.kick_drift_width, t.kick_drift_blocks) for t in arr]


def request_footprint(params) -> int:
    return load().vlasov_request_footprint(C.byref(to_params(params, 0)))


def device_copy(dst, src, nbytes: int, stream=None):
    """Library streaming copy between two device tensors (bandwidth ceiling)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    check(load().vlasov_device_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), int(nbytes),
                                    C.c_void_p(s.cuda_stream)))
