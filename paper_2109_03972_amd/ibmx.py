"""Thin ctypes binding of libibmx.so (include/ibmx.h).

Only argument marshalling lives here: tensors provide device memory through
``data_ptr()`` and the stream is torch's current HIP stream.  Every step of
the forcing loop and the pair pass runs in the library's HIP kernels; if the
library is missing the calls raise instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibmx.so")

OK, EINVAL, EDOMAIN, ENOMEM, EDEVICE, ESTATE, ECAPACITY, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
F64, F32 = 0, 1
RESERVE_BACKWARD, RESERVE_FLUID = 1, 2

# every entry point declared in include/ibmx.h
API = (
    "ibmx_plan_create", "ibmx_plan_destroy", "ibmx_plan_set_markers", "ibmx_plan_set_params",
    "ibmx_plan_set_stream", "ibmx_plan_set_tiles", "ibmx_plan_status", "ibmx_plan_stats",
    "ibmx_plan_profile", "ibmx_plan_set_launch", "ibmx_plan_reserve",
    "ibmx_forcing", "ibmx_forcing_graph",
    "ibmx_forcing_backward", "ibmx_pairs", "ibmx_tune", "ibmx_particle_integrals",
    "ibmx_grid_mean", "ibmx_particle_substeps", "ibmx_project", "ibmx_fluid_predictor",
    "ibmx_fluid_helmholtz", "ibmx_grid_mean_noalloc", "ibmx_status_string", "ibmx_version",
)

HIST = 4   # rows of a contact history array (IBMX_HIST)


class IbmxError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = code
        super().__init__(f"{where}: ibmx status {code} ({status_string(code)})")


class ibmx_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("periodic", ctypes.c_int32 * 3),
                ("h", ctypes.c_double), ("origin", ctypes.c_double * 3)]


class ibmx_params(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("n_iter", ctypes.c_int32),
                ("two_alpha_dt", ctypes.c_double), ("rho_f", ctypes.c_double),
                ("nu_f", ctypes.c_double), ("eps_sep", ctypes.c_double),
                ("lub_C", ctypes.c_double), ("zeta_min_factor", ctypes.c_double),
                ("e_dry", ctypes.c_double), ("T_c", ctypes.c_double), ("mu_s", ctypes.c_double),
                ("mu_k", ctypes.c_double), ("nu_poi", ctypes.c_double), ("dt", ctypes.c_double),
                ("gap_cut", ctypes.c_double), ("disable_mode", ctypes.c_int32),
                ("normal_model", ctypes.c_int32), ("disable_seed", ctypes.c_uint64),
                ("St_crit", ctypes.c_double), ("gravity", ctypes.c_double * 3),
                ("kn_grav_eps", ctypes.c_double), ("st_switch", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class ibmx_stats(ctypes.Structure):
    _fields_ = [("n_markers", ctypes.c_int64), ("n_active", ctypes.c_int64),
                ("shell_nodes", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("halo_entries", ctypes.c_int64), ("tile", ctypes.c_int32 * 3),
                ("block", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("kernel_ms", ctypes.c_double * 8),
                ("kernel_launches", ctypes.c_int64 * 8)]

KERNEL_CLASSES = ("geometry", "interp", "spread", "backward", "pairs", "other", "ftot", "graph")


_lib = None


def lib():
    """Load libibmx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, St = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
        L.ibmx_plan_create.restype = St
        L.ibmx_plan_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(ibmx_grid),
                                       ctypes.POINTER(ibmx_params), i32, P, St, P]
        L.ibmx_plan_destroy.restype = St
        L.ibmx_plan_destroy.argtypes = [P]
        L.ibmx_plan_set_markers.restype = St
        L.ibmx_plan_set_markers.argtypes = [P, P, P]
        L.ibmx_plan_set_params.restype = St
        L.ibmx_plan_set_params.argtypes = [P, ctypes.POINTER(ibmx_params)]
        L.ibmx_plan_set_stream.restype = St
        L.ibmx_plan_set_stream.argtypes = [P, P]
        L.ibmx_plan_set_tiles.restype = St
        L.ibmx_plan_set_tiles.argtypes = [P, i32, i32, i32]
        L.ibmx_plan_status.restype = St
        L.ibmx_plan_status.argtypes = [P]
        L.ibmx_plan_stats.restype = St
        L.ibmx_plan_stats.argtypes = [P, ctypes.POINTER(ibmx_stats)]
        L.ibmx_plan_profile.restype = St
        L.ibmx_plan_profile.argtypes = [P, i32]
        L.ibmx_plan_set_launch.restype = St
        L.ibmx_plan_set_launch.argtypes = [P, i32, i32]
        L.ibmx_plan_reserve.restype = St
        L.ibmx_plan_reserve.argtypes = [P, i32, i32, i32, i32]
        L.ibmx_forcing.restype = St
        L.ibmx_forcing.argtypes = [P] * 11
        L.ibmx_forcing_graph.restype = St
        L.ibmx_forcing_graph.argtypes = [P] * 11
        L.ibmx_forcing_backward.restype = St
        L.ibmx_forcing_backward.argtypes = [P] * 14
        L.ibmx_pairs.restype = St
        L.ibmx_pairs.argtypes = [P, P, P, ctypes.c_double, P, P, P, i32, P, P, i32, P, P, P, i32,
                                 P, P, P, P, i32, P, P, P, i32, P, P, P, P]
        L.ibmx_tune.restype = St
        L.ibmx_tune.argtypes = [P] * 7
        L.ibmx_particle_integrals.restype = St
        L.ibmx_particle_integrals.argtypes = [P] * 7
        L.ibmx_grid_mean.restype = St
        L.ibmx_grid_mean.argtypes = [P] * 3
        L.ibmx_grid_mean_noalloc.restype = St
        L.ibmx_grid_mean_noalloc.argtypes = [P, ctypes.c_int64, St, P, P]
        L.ibmx_fluid_predictor.restype = St
        L.ibmx_fluid_predictor.argtypes = [P, P, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double]
        L.ibmx_fluid_helmholtz.restype = St
        L.ibmx_fluid_helmholtz.argtypes = [P, P, P, P, P, ctypes.c_double, ctypes.c_double]
        L.ibmx_project.restype = St
        L.ibmx_project.argtypes = [P, P, P, P, P, ctypes.c_double]
        L.ibmx_particle_substeps.restype = St
        L.ibmx_particle_substeps.argtypes = [P, ctypes.c_double, i32, P, P, P, P, P, P, P, P, i32,
                                             P, i32, P, P, P, P, P]
        L.ibmx_status_string.restype = ctypes.c_char_p
        L.ibmx_status_string.argtypes = [St]
        L.ibmx_version.restype = ctypes.c_char_p
        L.ibmx_version.argtypes = []
        _lib = L
    return _lib


def status_string(code: int) -> str:
    try:
        return lib().ibmx_status_string(int(code)).decode()
    except Exception:  # library missing: still format the error
        return "?"


def version() -> str:
    return lib().ibmx_version().decode()


def _check(code: int, where: str):
    if code != OK:
        raise IbmxError(code, where)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_params(prm: Dict) -> ibmx_params:
    p = ibmx_params()
    p.kernel = int(prm.get("kernel", 3))
    p.n_iter = int(prm["n_iter"])
    p.two_alpha_dt = float(prm["c"])
    for k in ("rho_f", "nu_f", "eps_sep", "lub_C", "zeta_min_factor", "e_dry", "T_c", "mu_s",
              "mu_k", "nu_poi", "dt", "gap_cut"):
        setattr(p, k, float(prm[k]))
    p.disable_mode = int(prm.get("disable_mode", 0))
    p.normal_model = int(prm.get("normal_model", 0))
    p.disable_seed = int(prm.get("disable_seed", 0)) & 0xFFFFFFFFFFFFFFFF
    p.St_crit = float(prm.get("St_crit", 5.0))
    g = prm.get("gravity", (0.0, 0.0, 0.0))
    for a in range(3):
        p.gravity[a] = float(g[a])
    p.kn_grav_eps = float(prm.get("kn_grav_eps", 1e-3))
    p.st_switch = int(prm.get("st_switch", 0))
    p.reserved = 0
    return p


def make_grid(n, h, origin, periodic) -> ibmx_grid:
    g = ibmx_grid()
    for a in range(3):
        g.n[a] = int(n[a])
        g.periodic[a] = int(periodic[a])
        g.origin[a] = float(origin[a])
    g.h = float(h)
    return g


def _want(t, dtype, shape, name):
    import torch
    if t is None:
        return
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Plan:
    """Owns an ibmx_plan: grid, parameters, marker layout and workspace."""

    def __init__(self, n, h, origin, periodic, params: Dict, moff, precision: str = "f64"):
        import torch
        self.n = tuple(int(v) for v in n)
        self.h = float(h)
        self.origin = tuple(float(v) for v in origin)
        self.periodic = tuple(int(v) for v in periodic)
        self.params = dict(params)
        self.moff = np.ascontiguousarray(moff, dtype=np.int32)
        self.np = int(self.moff.shape[0] - 1)
        self.nm = int(self.moff[-1]) if self.np > 0 else 0
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self._grid = make_grid(self.n, self.h, self.origin, self.periodic)
        self._prm = make_params(self.params)
        h_ = ctypes.c_void_p()
        st = lib().ibmx_plan_create(ctypes.byref(h_), ctypes.byref(self._grid), ctypes.byref(self._prm),
                                    self.np, self.moff.ctypes.data_as(ctypes.c_void_p),
                                    F64 if precision == "f64" else F32, _stream())
        _check(st, "ibmx_plan_create")
        self.handle = h_
        self._markers = None
        # workspace reserved with ibmx_plan_reserve: pair, wall, cell
        # capacities and flags
        self._res = [0, 0, 0, 0]

    @classmethod
    def from_case(cls, case, precision="f64", params=None):
        return cls(case.n, case.h, case.origin, case.periodic, params or case.params, case.moff,
                   precision)

    # -- life cycle ----------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().ibmx_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        lib().ibmx_plan_set_stream(self.handle, _stream())

    def set_markers(self, body, dV):
        import torch
        _want(body, torch.float64, (3, self.nm), "body")
        _want(dV, torch.float64, (self.np,), "dV")
        self._markers = (body, dV)       # keep the memory alive
        _check(lib().ibmx_plan_set_markers(self.handle, _ptr(body), _ptr(dV)), "ibmx_plan_set_markers")

    def set_params(self, params: Dict):
        self.params = dict(params)
        self._prm = make_params(self.params)
        _check(lib().ibmx_plan_set_params(self.handle, ctypes.byref(self._prm)), "ibmx_plan_set_params")

    def set_tiles(self, tx: int, ty: int, tz: int):
        _check(lib().ibmx_plan_set_tiles(self.handle, int(tx), int(ty), int(tz)),
               "ibmx_plan_set_tiles")

    def reserve(self, pair_cap: int = 0, wall_cap: int = 0, cell_cap: int = 0,
                backward: bool = False, fluid: bool = False):
        """ibmx_plan_reserve: grow the workspace of the pair pass, the
        sub-stepping, the adjoint and the fluid solves (synchronises; call it
        outside graph capture)."""
        flags = (RESERVE_BACKWARD if backward else 0) | (RESERVE_FLUID if fluid else 0)
        _check(lib().ibmx_plan_reserve(self.handle, int(pair_cap), int(wall_cap), int(cell_cap),
                                       flags), "ibmx_plan_reserve")
        r = self._res
        self._res = [max(r[0], int(pair_cap)), max(r[1], int(wall_cap)), max(r[2], int(cell_cap)),
                     r[3] | flags]

    def _ensure(self, pair_cap=0, wall_cap=0, cell_cap=0, flags=0):
        """Reserve what a call needs beyond the current reservation."""
        r = self._res
        if pair_cap > r[0] or wall_cap > r[1] or cell_cap > r[2] or (flags & ~r[3]):
            self.reserve(max(r[0], pair_cap), max(r[1], wall_cap), max(r[2], cell_cap),
                         backward=bool((flags | r[3]) & RESERVE_BACKWARD),
                         fluid=bool((flags | r[3]) & RESERVE_FLUID))

    def _ensure_fluid(self):
        """Reserve the solver workspace before the first solve; on grids the
        solves do not take, leave it to the call to report EUNSUPPORTED."""
        if self._res[3] & RESERVE_FLUID:
            return
        try:
            self._ensure(flags=RESERVE_FLUID)
        except IbmxError as e:
            if e.code != EUNSUPPORTED:
                raise

    def set_launch(self, block: int = 256, persistent: bool = False):
        _check(lib().ibmx_plan_set_launch(self.handle, int(block), int(persistent)),
               "ibmx_plan_set_launch")

    def status(self) -> int:
        return int(lib().ibmx_plan_status(self.handle))

    def check(self, where="ibmx"):
        _check(self.status(), where)

    def stats(self) -> Dict:
        s = ibmx_stats()
        _check(lib().ibmx_plan_stats(self.handle, ctypes.byref(s)), "ibmx_plan_stats")
        return dict(n_markers=s.n_markers, n_active=s.n_active, shell_nodes=s.shell_nodes,
                    tiles=s.tiles, halo_entries=s.halo_entries, tile=tuple(s.tile), block=s.block,
                    persistent=s.persistent,
                    kernel_ms={k: s.kernel_ms[i] for i, k in enumerate(KERNEL_CLASSES)},
                    kernel_launches={k: s.kernel_launches[i] for i, k in enumerate(KERNEL_CLASSES)})

    def profile(self, enable: bool = True):
        _check(lib().ibmx_plan_profile(self.handle, 1 if enable else 0), "ibmx_plan_profile")

    # -- compute calls ---------------------------------------------------------
    def forcing(self, u, f_tot, xp, up, wp, mask=None, S=None, T=None, resid=None, U_debug=None,
                graph=False):
        """ibmx_forcing (ibmx_forcing_graph with graph=True): updates u in
        place, accumulates into f_tot, returns (S, T)."""
        import torch
        grid_shape = (3, self.n[2], self.n[1], self.n[0])
        _want(u, self.dtype, grid_shape, "u")
        _want(f_tot, self.dtype, grid_shape, "f_tot")
        for t, nme in ((xp, "xp"), (up, "up"), (wp, "wp")):
            _want(t, torch.float64, (3, self.np), nme)
        _want(mask, torch.uint8, (self.nm,), "mask")
        dev = u.device
        if S is None:
            S = torch.empty((3, self.np), dtype=torch.float64, device=dev)
        if T is None:
            T = torch.empty((3, self.np), dtype=torch.float64, device=dev)
        _want(S, torch.float64, (3, self.np), "S")
        _want(T, torch.float64, (3, self.np), "T")
        _want(resid, torch.float64, (int(self.params["n_iter"]) + 1,), "resid")
        _want(U_debug, self.dtype, (int(self.params["n_iter"]), 3, self.nm), "U_debug")
        self._sync_stream()
        fn = lib().ibmx_forcing_graph if graph else lib().ibmx_forcing
        st = fn(self.handle, _ptr(u), _ptr(f_tot), _ptr(xp), _ptr(up), _ptr(wp), _ptr(mask),
                _ptr(S), _ptr(T), _ptr(resid), _ptr(U_debug))
        _check(st, "ibmx_forcing_graph" if graph else "ibmx_forcing")
        return S, T

    def forcing_backward(self, u0, xp, up, wp, mask, g_f, g_u, g_S, g_T, gu0=None):
        import torch
        grid_shape = (3, self.n[2], self.n[1], self.n[0])
        _want(u0, self.dtype, grid_shape, "u0")
        _want(g_f, self.dtype, grid_shape, "g_f")
        _want(g_u, self.dtype, grid_shape, "g_u")
        _want(g_S, torch.float64, (3, self.np), "g_S")
        _want(g_T, torch.float64, (3, self.np), "g_T")
        _want(mask, torch.uint8, (self.nm,), "mask")
        dev = u0.device
        self._ensure(flags=RESERVE_BACKWARD)
        if gu0 is None:
            gu0 = torch.empty(grid_shape, dtype=self.dtype, device=dev)
        gxp = torch.empty((3, self.np), dtype=torch.float64, device=dev)
        gup = torch.empty_like(gxp)
        gwp = torch.empty_like(gxp)
        self._sync_stream()
        st = lib().ibmx_forcing_backward(self.handle, _ptr(u0), _ptr(xp), _ptr(up), _ptr(wp),
                                         _ptr(mask), _ptr(g_f), _ptr(g_u), _ptr(g_S), _ptr(g_T),
                                         _ptr(gu0), _ptr(gxp), _ptr(gup), _ptr(gwp))
        _check(st, "ibmx_forcing_backward")
        return gu0, gxp, gup, gwp

    def pairs(self, xp, radius, mass, up, wp, prev=None, pair_cap=None, wall_cap=None,
              mask=None, cell_cap=None, radius_max=None):
        """ibmx_pairs: returns a dict of device tensors (lists are trimmed
        after a synchronising read of the counts)."""
        import torch
        dev = xp.device
        for t, nme in ((xp, "xp"), (up, "up"), (wp, "wp")):
            _want(t, torch.float64, (3, self.np), nme)
        _want(radius, torch.float64, (self.np,), "radius")
        _want(mass, torch.float64, (self.np,), "mass")
        if radius_max is None:
            if getattr(self, "_rmax", None) is None or self._rmax[0] is not radius:
                self._rmax = (radius, float(radius.max().item()) if self.np > 0 else 1.0)
            radius_max = self._rmax[1]
        pair_cap = int(pair_cap or max(64, 16 * self.np))
        wall_cap = int(wall_cap or max(64, 2 * self.np))
        cell_cap = int(cell_cap or (1 << 20))
        self._ensure(pair_cap, wall_cap, cell_cap)
        i32, f64 = torch.int32, torch.float64
        cell_start = torch.empty(cell_cap, dtype=i32, device=dev)
        cellp = torch.empty(max(self.np, 1), dtype=i32, device=dev)
        pairs = torch.empty((2, pair_cap), dtype=i32, device=dev)
        pgap = torch.empty(pair_cap, dtype=f64, device=dev)
        hist = torch.empty((HIST, pair_cap), dtype=f64, device=dev)
        walls = torch.empty((2, wall_cap), dtype=i32, device=dev)
        wgap = torch.empty(wall_cap, dtype=f64, device=dev)
        whist = torch.empty((HIST, wall_cap), dtype=f64, device=dev)
        counts = torch.zeros(2, dtype=i32, device=dev)
        Fc = torch.empty((3, self.np), dtype=f64, device=dev)
        Tc = torch.empty_like(Fc)
        if mask is None:
            mask = torch.empty(max(self.nm, 1), dtype=torch.uint8, device=dev)
        if prev is None:
            pin = torch.zeros((2, 1), dtype=i32, device=dev)
            hin = torch.zeros((HIST, 1), dtype=f64, device=dev)
            win = torch.zeros((2, 1), dtype=i32, device=dev)
            whin = torch.zeros((HIST, 1), dtype=f64, device=dev)
            n_in, nw_in = 0, 0
        else:
            pin, hin = prev["pairs"].contiguous(), prev["hist"].contiguous()
            win, whin = prev["walls"].contiguous(), prev["whist"].contiguous()
            n_in, nw_in = int(pin.shape[1]), int(win.shape[1])
            _want(hin, f64, (HIST, n_in), "prev hist")
            _want(whin, f64, (HIST, nw_in), "prev whist")
        self._sync_stream()
        st = lib().ibmx_pairs(self.handle, _ptr(xp), _ptr(radius), float(radius_max), _ptr(mass),
                              _ptr(up), _ptr(wp),
                              n_in, _ptr(pin), _ptr(hin), nw_in, _ptr(win), _ptr(whin),
                              _ptr(cell_start), cell_cap, _ptr(cellp), _ptr(pairs), _ptr(pgap),
                              _ptr(hist), pair_cap, _ptr(walls), _ptr(wgap), _ptr(whist), wall_cap,
                              _ptr(counts), _ptr(Fc), _ptr(Tc), _ptr(mask) if self.nm > 0 else None)
        _check(st, "ibmx_pairs")
        return dict(cell_start=cell_start, cell_particles=cellp, pairs=pairs, gap=pgap, hist=hist,
                    walls=walls, wgap=wgap, whist=whist, counts=counts, Fc=Fc, Tc=Tc, mask=mask,
                    pair_cap=pair_cap, wall_cap=wall_cap)

    def particle_substeps(self, dt_total, n_sub, xp, up, wp, radius, mass, lists, hist, whist,
                          Fh=None, Th=None, want_forces=True):
        """ibmx_particle_substeps: advances xp, up, wp (double[3][np] device
        tensors, in place) over the contact lists of a pairs() result
        (``lists``: its pairs, walls, counts and caps); ``hist``/``whist``
        double[4][cap] are updated in place.  Returns (Fc, Tc) at the final
        state, or None."""
        import torch
        f64 = torch.float64
        for t, nme in ((xp, "xp"), (up, "up"), (wp, "wp")):
            _want(t, f64, (3, self.np), nme)
        _want(radius, f64, (self.np,), "radius")
        _want(mass, f64, (self.np,), "mass")
        _want(Fh, f64, (3, self.np), "Fh")
        _want(Th, f64, (3, self.np), "Th")
        pc, wc = int(lists["pair_cap"]), int(lists["wall_cap"])
        self._ensure(pc, wc)
        _want(lists["pairs"], torch.int32, (2, pc), "pairs")
        _want(lists["walls"], torch.int32, (2, wc), "walls")
        _want(lists["counts"], torch.int32, (2,), "counts")
        _want(hist, f64, (HIST, pc), "hist")
        _want(whist, f64, (HIST, wc), "whist")
        Fc = Tc = None
        if want_forces:
            Fc = torch.empty((3, self.np), dtype=f64, device=xp.device)
            Tc = torch.empty_like(Fc)
        self._sync_stream()
        st = lib().ibmx_particle_substeps(self.handle, float(dt_total), int(n_sub), _ptr(xp),
                                          _ptr(up), _ptr(wp), _ptr(radius), _ptr(mass), _ptr(Fh),
                                          _ptr(Th), _ptr(lists["counts"]), pc, _ptr(lists["pairs"]),
                                          wc, _ptr(lists["walls"]), _ptr(hist), _ptr(whist),
                                          _ptr(Fc), _ptr(Tc))
        _check(st, "ibmx_particle_substeps")
        return (Fc, Tc) if want_forces else None

    def fluid_predictor(self, u, N, P, dt, gamma, zeta, u_out=None, lapnu=None):
        """ibmx_fluid_predictor: returns (u~, lapnu); N is updated in place."""
        import torch
        shape = (self.n[2], self.n[1], self.n[0])
        for t, nme in ((u, "u"), (N, "N"), (u_out, "u_out"), (lapnu, "lapnu")):
            _want(t, self.dtype, (3,) + shape, nme)
        _want(P, self.dtype, shape, "P")
        u_out = torch.empty_like(u) if u_out is None else u_out
        lapnu = torch.empty_like(u) if lapnu is None else lapnu
        self._sync_stream()
        st = lib().ibmx_fluid_predictor(self.handle, _ptr(u), _ptr(u_out), _ptr(N), _ptr(lapnu),
                                        _ptr(P), float(dt), float(gamma), float(zeta))
        _check(st, "ibmx_fluid_predictor")
        return u_out, lapnu

    def fluid_helmholtz(self, u, lapnu, P, dt, theta=0.0, fbar=None):
        """ibmx_fluid_helmholtz: u (forced velocity) is overwritten by u*."""
        import torch
        shape = (self.n[2], self.n[1], self.n[0])
        _want(u, self.dtype, (3,) + shape, "u")
        _want(lapnu, self.dtype, (3,) + shape, "lapnu")
        _want(P, self.dtype, shape, "P")
        _want(fbar, torch.float64, (3,), "fbar")
        self._ensure_fluid()
        self._sync_stream()
        st = lib().ibmx_fluid_helmholtz(self.handle, _ptr(u), _ptr(lapnu), _ptr(P), _ptr(fbar),
                                        float(dt), float(theta))
        _check(st, "ibmx_fluid_helmholtz")

    def project(self, u, P, theta=0.0, want_phi=True):
        """ibmx_project: projects u (the plan's precision, [3][nz][ny][nx]) in
        place and updates P ([nz][ny][nx]) in place; returns (uf, phi)."""
        import torch
        shape = (self.n[2], self.n[1], self.n[0])
        _want(u, self.dtype, (3,) + shape, "u")
        _want(P, self.dtype, shape, "P")
        uf = torch.empty_like(u)
        phi = torch.empty_like(P) if want_phi else None
        self._ensure_fluid()
        self._sync_stream()
        st = lib().ibmx_project(self.handle, _ptr(u), _ptr(uf), _ptr(P), _ptr(phi), float(theta))
        _check(st, "ibmx_project")
        return uf, phi

    def particle_integrals(self, u, xp, radius, alpha=None):
        """ibmx_particle_integrals: returns (Iu, Ir), double[3][np]; fills the
        optional alpha grid (the plan's precision, [nz][ny][nx])."""
        import torch
        grid_shape = (3, self.n[2], self.n[1], self.n[0])
        _want(u, self.dtype, grid_shape, "u")
        _want(xp, torch.float64, (3, self.np), "xp")
        _want(radius, torch.float64, (self.np,), "radius")
        _want(alpha, self.dtype, grid_shape[1:], "alpha")
        Iu = torch.empty((3, self.np), dtype=torch.float64, device=u.device)
        Ir = torch.empty_like(Iu)
        self._sync_stream()
        st = lib().ibmx_particle_integrals(self.handle, _ptr(u), _ptr(xp), _ptr(radius), _ptr(Iu),
                                           _ptr(Ir), _ptr(alpha))
        _check(st, "ibmx_particle_integrals")
        return Iu, Ir

    def grid_mean(self, f):
        """ibmx_grid_mean: per-component volume average (double[3] on the device)."""
        import torch
        _want(f, self.dtype, (3, self.n[2], self.n[1], self.n[0]), "f")
        mean = torch.empty(3, dtype=torch.float64, device=f.device)
        self._sync_stream()
        _check(lib().ibmx_grid_mean(self.handle, _ptr(f), _ptr(mean)), "ibmx_grid_mean")
        return mean

    def tune(self, u, f_tot, xp, up, wp, mask=None):
        self._sync_stream()
        st = lib().ibmx_tune(self.handle, _ptr(u), _ptr(f_tot), _ptr(xp), _ptr(up), _ptr(wp),
                             _ptr(mask))
        _check(st, "ibmx_tune")
        return self.stats()


def grid_mean_noalloc(f, mean=None):
    """ibmx_grid_mean_noalloc: per-component mean of a [3][...] device
    tensor (float32 or float64) without a plan; returns double[3] on the
    device (``mean`` is written if given)."""
    import torch
    if not isinstance(f, torch.Tensor) or not f.is_cuda or not f.is_contiguous():
        raise TypeError("f must be a contiguous device tensor")
    if f.dtype not in (torch.float32, torch.float64) or f.dim() < 1 or f.shape[0] != 3:
        raise ValueError("f must be float32 or float64 with 3 components in its first dimension")
    if mean is None:
        mean = torch.empty(3, dtype=torch.float64, device=f.device)
    _want(mean, torch.float64, (3,), "mean")
    prec = F64 if f.dtype == torch.float64 else F32
    _check(lib().ibmx_grid_mean_noalloc(_ptr(f), f.numel() // 3, prec, _ptr(mean), _stream()),
           "ibmx_grid_mean_noalloc")
    return mean


def trim_pairs(res: Dict) -> Dict:
    """Host-side view of a pairs() result with the lists cut to their counts."""
    cnt = res["counts"].cpu().numpy()
    k, kw = int(cnt[0]), int(cnt[1])
    return dict(pairs=res["pairs"][:, :k], gap=res["gap"][:k], hist=res["hist"][:, :k],
                walls=res["walls"][:, :kw], wgap=res["wgap"][:kw], whist=res["whist"][:, :kw],
                npairs=k, nwall=kw)


def _autograd_function():
    import torch

    class IBMForcing(torch.autograd.Function):
        """Differentiable forcing loop: (u0, x_p, u_p, omega_p) ->
        (u^n, f_tot, S, T).  The backward pass is ibmx_forcing_backward,
        which replays the passes on the device; the mask, body offsets and
        marker volumes are held fixed."""

        @staticmethod
        def forward(ctx, plan, u0, xp, up, wp, mask):
            u = u0.detach().clone()
            f = torch.zeros_like(u)
            S, T = plan.forcing(u, f, xp.detach(), up.detach(), wp.detach(), mask=mask)
            ctx.plan = plan
            ctx.save_for_backward(u0.detach(), xp.detach(), up.detach(), wp.detach())
            ctx.mask = mask
            return u, f, S, T

        @staticmethod
        def backward(ctx, g_u, g_f, g_S, g_T):
            u0, xp, up, wp = ctx.saved_tensors

            def cont(t):
                return None if t is None else t.contiguous()

            gu0, gxp, gup, gwp = ctx.plan.forcing_backward(
                u0, xp, up, wp, ctx.mask, cont(g_f), cont(g_u), cont(g_S), cont(g_T))
            return None, gu0, gxp, gup, gwp, None

    return IBMForcing


_IBM_FORCING = None


def forcing_autograd(plan: "Plan", u0, xp, up, wp, mask=None):
    """Autograd entry: returns (u, f_tot, S, T) for a forcing call starting
    from u0 with f_tot = 0; gradients flow to u0, xp, up and wp."""
    global _IBM_FORCING
    if _IBM_FORCING is None:
        _IBM_FORCING = _autograd_function()
    return _IBM_FORCING.apply(plan, u0, xp, up, wp, mask)
