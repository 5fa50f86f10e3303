"""Plain FP64 CPU oracle of the forcing loop and the pair pass.

TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the HIP library.  ``build()`` compiles ``ibmx_oracle.c`` with gcc
(-O2, no FMA contraction) into ``libibmx_oracle.so`` next to this file.
"""
from __future__ import annotations

import ctypes
import functools
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ibmx_oracle.c")
# IBMX_ORACLE_SANITIZE=1 selects a build with AddressSanitizer and
# UndefinedBehaviorSanitizer (the process must preload the ASan runtime)
_SANITIZE = os.environ.get("IBMX_ORACLE_SANITIZE", "") == "1"
_LIB = os.path.join(_HERE, "libibmx_oracle_san.so" if _SANITIZE else "libibmx_oracle.so")
_lib = None

OK, EINVAL, EDOMAIN, ECAPACITY = 0, -1, -2, -6


def build(force: bool = True) -> str:
    """Compile the oracle (gcc -O2 -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        san = (["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                "-fno-omit-frame-pointer", "-g"] if _SANITIZE else [])
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                               "-D_DEFAULT_SOURCE", "-fPIC", "-shared", *san, "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        d, i, u64 = ctypes.c_double, ctypes.c_int, ctypes.c_uint64
        P = ctypes.c_void_p
        for f in ("ref_phi3", "ref_dphi3", "ref_phi4", "ref_dphi4"):
            getattr(L, f).restype = d
            getattr(L, f).argtypes = [d]
        L.ref_splitmix64.restype = u64
        L.ref_splitmix64.argtypes = [u64]
        L.ref_forcing.restype = i
        L.ref_forcing.argtypes = [P, d, P, P, i, i, d, i, i, P, P, P, P, P, P, P, P, P, P, P, P, P]
        L.ref_forcing_adjoint.restype = i
        L.ref_forcing_adjoint.argtypes = [P, d, P, P, i, i, d, i, P, P, P, P, P, P, P, P,
                                          P, P, P, P, P, P, P, P]
        L.ref_cell_list.restype = i
        L.ref_cell_list.argtypes = [P, d, P, P, i, P, P, d, P, i, P, P, P]
        L.ref_pairs_brute.restype = i
        L.ref_pairs_brute.argtypes = [P, d, P, P, i, P, P, d, i, P, P, P]
        L.ref_walls.restype = i
        L.ref_walls.argtypes = [P, d, P, P, i, P, P, d, i, P, P, P]
        L.ref_actm_coefficients.restype = i
        L.ref_actm_coefficients.argtypes = [d, d, P, P]
        L.ref_particle_substeps.restype = i
        L.ref_particle_substeps.argtypes = [P, d, P, P, i, P, P, P, P, P, P, P, P, d, i, i, P, i,
                                            P, P, P, P, P]
        L.ref_pair_forces.restype = i
        L.ref_pair_forces.argtypes = [P, d, P, P, i, P, P, P, P, P, P, i, P, i, P,
                                      i, P, P, i, P, P, P, P, P, P]
        L.ref_marker_mask.restype = i
        L.ref_marker_mask.argtypes = [P, d, P, P, i, P, P, P, P, d, i, u64, i, P, P, i, P, P, P]
        L.ref_particle_integrals.restype = i
        L.ref_particle_integrals.argtypes = [P, d, P, P, i, P, P, P, P, P, P]
        L.ref_cell_alpha.restype = d
        L.ref_cell_alpha.argtypes = [P, d, d]
        L.ref_grid_mean.restype = i
        L.ref_grid_mean.argtypes = [P, P, P]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _grid(case):
    return (np.asarray(case.n, dtype=np.int32), float(case.h),
            np.asarray(case.origin, dtype=np.float64), np.asarray(case.periodic, dtype=np.int32))


def phi3(r: float) -> float:
    return lib().ref_phi3(float(r))


def dphi3(r: float) -> float:
    return lib().ref_dphi3(float(r))


def phi4(r: float) -> float:
    return lib().ref_phi4(float(r))


def dphi4(r: float) -> float:
    return lib().ref_dphi4(float(r))


def splitmix64(x: int) -> int:
    return int(lib().ref_splitmix64(int(x) & 0xFFFFFFFFFFFFFFFF))


def forcing(case, u0=None, f_tot=None, mask=None, xp=None, up=None, wp=None,
            n_iter=None, c=None, kernel=None, final_resid=True, want_U=False):
    """Run the outer forcing loop.  Returns dict(u, f_tot, S, T, resid, U)."""
    n, h, origin, per = _grid(case)
    prm = case.params
    n_iter = int(prm["n_iter"] if n_iter is None else n_iter)
    c = float(prm["c"] if c is None else c)
    kernel = int(prm.get("kernel", 3) if kernel is None else kernel)
    u = _f64(case.u0 if u0 is None else u0).copy()
    ft = np.zeros_like(u) if f_tot is None else _f64(f_tot).copy()
    npart, nm = case.np_, case.nm
    S = np.zeros((3, npart))
    T = np.zeros((3, npart))
    resid = np.zeros(n_iter + 1)
    U = np.zeros((n_iter, 3, nm)) if want_U else None
    xp_ = _f64(case.xp if xp is None else xp)
    up_ = _f64(case.up if up is None else up)
    wp_ = _f64(case.wp if wp is None else wp)
    moff, body, dV = _i32(case.moff), _f64(case.body), _f64(case.dV)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    st = lib().ref_forcing(_p(n), h, _p(origin), _p(per), kernel, n_iter, c, int(final_resid),
                           npart, _p(moff), _p(body), _p(dV), _p(xp_), _p(up_), _p(wp_), _p(mk),
                           _p(u), _p(ft), _p(S), _p(T), _p(resid), _p(U))
    if st != OK:
        raise OracleError(st)
    return dict(u=u, f_tot=ft, S=S, T=T, resid=resid, U=U)


def forcing_adjoint(case, u0=None, mask=None, g_f=None, g_u=None, g_S=None, g_T=None,
                    xp=None, up=None, wp=None, n_iter=None, c=None, kernel=None):
    n, h, origin, per = _grid(case)
    prm = case.params
    n_iter = int(prm["n_iter"] if n_iter is None else n_iter)
    c = float(prm["c"] if c is None else c)
    kernel = int(prm.get("kernel", 3) if kernel is None else kernel)
    u0_ = _f64(case.u0 if u0 is None else u0)
    npart = case.np_
    gu0 = np.zeros_like(u0_)
    gxp = np.zeros((3, npart))
    gup = np.zeros((3, npart))
    gwp = np.zeros((3, npart))
    xp_ = _f64(case.xp if xp is None else xp)
    up_ = _f64(case.up if up is None else up)
    wp_ = _f64(case.wp if wp is None else wp)
    moff, body, dV = _i32(case.moff), _f64(case.body), _f64(case.dV)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    args = [None if a is None else _f64(a) for a in (g_f, g_u, g_S, g_T)]
    st = lib().ref_forcing_adjoint(_p(n), h, _p(origin), _p(per), kernel, n_iter, c, npart,
                                   _p(moff), _p(body), _p(dV), _p(xp_), _p(up_), _p(wp_), _p(mk),
                                   _p(u0_), *[_p(a) for a in args],
                                   _p(gu0), _p(gxp), _p(gup), _p(gwp))
    if st != OK:
        raise OracleError(st)
    return dict(gu0=gu0, gxp=gxp, gup=gup, gwp=gwp)


def cell_list(case, xp=None, gap_cut=None):
    n, h, origin, per = _grid(case)
    gap_cut = float(case.params["gap_cut"] if gap_cut is None else gap_cut)
    xp_ = _f64(case.xp if xp is None else xp)
    npart = case.np_
    nc = np.zeros(3, dtype=np.int32)
    cap = 1 << 22
    cell_of = np.zeros(max(npart, 1), dtype=np.int32)
    cell_start = np.zeros(cap + 1, dtype=np.int32)
    cellp = np.zeros(max(npart, 1), dtype=np.int32)
    st = lib().ref_cell_list(_p(n), h, _p(origin), _p(per), npart, _p(xp_), _p(_f64(case.radius)),
                             gap_cut, _p(nc), cap, _p(cell_of), _p(cell_start), _p(cellp))
    if st != OK:
        raise OracleError(st)
    ncell = int(nc[0]) * int(nc[1]) * int(nc[2])
    return dict(nc=nc, cell_of=cell_of[:npart], cell_start=cell_start[:ncell + 1],
                cell_particles=cellp[:npart])


def pairs(case, xp=None, gap_cut=None, cap=None):
    n, h, origin, per = _grid(case)
    gap_cut = float(case.params["gap_cut"] if gap_cut is None else gap_cut)
    xp_ = _f64(case.xp if xp is None else xp)
    npart = case.np_
    cap = cap or max(16, 16 * npart)
    pr = np.zeros((2, cap), dtype=np.int32)
    gp = np.zeros(cap)
    cnt = np.zeros(1, dtype=np.int32)
    st = lib().ref_pairs_brute(_p(n), h, _p(origin), _p(per), npart, _p(xp_), _p(_f64(case.radius)),
                               gap_cut, cap, _p(pr), _p(gp), _p(cnt))
    if st != OK:
        raise OracleError(st)
    k = int(cnt[0])
    wl = np.zeros((2, cap), dtype=np.int32)
    wg = np.zeros(cap)
    wc = np.zeros(1, dtype=np.int32)
    st = lib().ref_walls(_p(n), h, _p(origin), _p(per), npart, _p(xp_), _p(_f64(case.radius)),
                         gap_cut, cap, _p(wl), _p(wg), _p(wc))
    if st != OK:
        raise OracleError(st)
    kw = int(wc[0])
    return dict(pairs=np.ascontiguousarray(pr[:, :k]), gap=gp[:k].copy(),
                walls=np.ascontiguousarray(wl[:, :kw]), wgap=wg[:kw].copy())


HIST = 4   # history rows per contact: tangential spring (3), impact speed


@functools.lru_cache(maxsize=None)
def actm_coefficients(e: float, p: float = 1.5):
    """(K, D) of the normal collision ODE in contact-time units (Sec. 2.2.7,
    eq. ode): z'' + D z' + K z^p = 0 closes at t = 1 with rebound -e."""
    K = ctypes.c_double()
    D = ctypes.c_double()
    st = lib().ref_actm_coefficients(float(e), float(p), ctypes.byref(K), ctypes.byref(D))
    if st != OK:
        raise OracleError(st)
    return K.value, D.value


def collision_params(prm) -> np.ndarray:
    model = int(prm.get("normal_model", 0))
    K, D = actm_coefficients(float(prm["e_dry"])) if model == 1 else (0.0, 0.0)
    g = prm.get("gravity", (0.0, 0.0, 0.0))
    return np.array([prm["rho_f"], prm["nu_f"], prm["eps_sep"], prm["lub_C"], prm["zeta_min_factor"],
                     prm["e_dry"], prm["T_c"], prm["mu_s"], prm["mu_k"], prm["nu_poi"], prm["dt"],
                     model, prm.get("St_crit", 5.0), prm.get("kn_grav_eps", 1e-3),
                     g[0], g[1], g[2], K, D, int(prm.get("st_switch", 0))],
                    dtype=np.float64)


def pair_forces(case, plist, xp=None, up=None, wp=None, prev=None, params=None):
    """Collision force/torque for the lists in ``plist`` (from ``pairs``).
    ``prev`` = dict(pairs, hist, walls, whist) of a previous call or None;
    histories are [4][n] (tangential spring, impact speed)."""
    n, h, origin, per = _grid(case)
    npart = case.np_
    xp_ = _f64(case.xp if xp is None else xp)
    up_ = _f64(case.up if up is None else up)
    wp_ = _f64(case.wp if wp is None else wp)
    cp = collision_params(params or case.params)
    pr = _i32(plist["pairs"])
    wl = _i32(plist["walls"])
    npairs, nwall = pr.shape[1], wl.shape[1]
    if prev is None:
        prev = dict(pairs=np.zeros((2, 0), np.int32), hist=np.zeros((HIST, 0)),
                    walls=np.zeros((2, 0), np.int32), whist=np.zeros((HIST, 0)))
    ppr, phs = _i32(prev["pairs"]), _f64(prev["hist"])
    pwl, pwh = _i32(prev["walls"]), _f64(prev["whist"])
    assert phs.shape[0] == HIST and pwh.shape[0] == HIST
    Fc = np.zeros((3, npart))
    Tc = np.zeros((3, npart))
    hist = np.zeros((HIST, npairs))
    whist = np.zeros((HIST, nwall))
    st = lib().ref_pair_forces(_p(n), h, _p(origin), _p(per), npart, _p(xp_), _p(_f64(case.radius)),
                               _p(_f64(case.mass)), _p(up_), _p(wp_), _p(cp),
                               npairs, _p(pr), nwall, _p(wl),
                               ppr.shape[1], _p(ppr), _p(phs), pwl.shape[1], _p(pwl), _p(pwh),
                               _p(Fc), _p(Tc), _p(hist), _p(whist))
    if st != OK:
        raise OracleError(st)
    return dict(Fc=Fc, Tc=Tc, hist=hist, whist=whist)


def particle_substeps(case, plist, dt_total, n_sub, Fh=None, Th=None, hist=None, whist=None,
                      xp=None, up=None, wp=None, params=None):
    """Advance (x_p, u_p, omega_p) by dt_total in n_sub Runge-Kutta
    sub-steps (Sec. 2.2.10) on the fixed lists ``plist``; histories aligned
    with the lists ([4][n], zero = no history).  Returns the new state, the
    committed histories and the collision force/torque at the final state."""
    n, h, origin, per = _grid(case)
    npart = case.np_
    xp_ = _f64(case.xp if xp is None else xp).copy()
    up_ = _f64(case.up if up is None else up).copy()
    wp_ = _f64(case.wp if wp is None else wp).copy()
    cp = collision_params(params or case.params)
    pr = _i32(plist["pairs"])
    wl = _i32(plist["walls"])
    npairs, nwall = pr.shape[1], wl.shape[1]
    hs = np.zeros((HIST, npairs)) if hist is None else _f64(hist).copy()
    wh = np.zeros((HIST, nwall)) if whist is None else _f64(whist).copy()
    assert hs.shape == (HIST, npairs) and wh.shape == (HIST, nwall)
    Fh_ = None if Fh is None else _f64(Fh)
    Th_ = None if Th is None else _f64(Th)
    Fc = np.zeros((3, npart))
    Tc = np.zeros((3, npart))
    st = lib().ref_particle_substeps(_p(n), h, _p(origin), _p(per), npart, _p(xp_), _p(up_), _p(wp_),
                                     _p(_f64(case.radius)), _p(_f64(case.mass)), _p(cp), _p(Fh_),
                                     _p(Th_), float(dt_total), int(n_sub), npairs, _p(pr), nwall,
                                     _p(wl), _p(hs), _p(wh), _p(Fc), _p(Tc))
    if st != OK:
        raise OracleError(st)
    return dict(xp=xp_, up=up_, wp=wp_, hist=hs, whist=wh, Fc=Fc, Tc=Tc)


def marker_mask(case, plist, xp=None, mode=None, seed=None, eps_sep=None):
    n, h, origin, per = _grid(case)
    prm = case.params
    mode = int(prm["disable_mode"] if mode is None else mode)
    seed = int(prm["disable_seed"] if seed is None else seed)
    eps = float(prm["eps_sep"] if eps_sep is None else eps_sep)
    xp_ = _f64(case.xp if xp is None else xp)
    mask = np.zeros(case.nm, dtype=np.uint8)
    pr, wl = _i32(plist["pairs"]), _i32(plist["walls"])
    st = lib().ref_marker_mask(_p(n), h, _p(origin), _p(per), case.np_, _p(_i32(case.moff)),
                               _p(_f64(case.body)), _p(xp_), _p(_f64(case.radius)), eps, mode,
                               seed & 0xFFFFFFFFFFFFFFFF, pr.shape[1], _p(pr), _p(_f64(plist["gap"])),
                               wl.shape[1], _p(wl), _p(_f64(plist["wgap"])), _p(mask))
    if st != OK:
        raise OracleError(st)
    return mask


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle returned status {code}")
        self.code = code


def particle_integrals(case, u=None, xp=None, radius=None, want_alpha=False):
    """Level-set volume fraction integrals of the fluid velocity over each
    particle: returns dict(Iu, Ir[, alpha])."""
    n, h, origin, per = _grid(case)
    u_ = _f64(case.u0 if u is None else u)
    xp_ = _f64(case.xp if xp is None else xp)
    rad = _f64(case.radius if radius is None else radius)
    npart = xp_.shape[1]
    Iu = np.zeros((3, npart))
    Ir = np.zeros((3, npart))
    alpha = np.zeros(u_.shape[1:]) if want_alpha else None
    st = lib().ref_particle_integrals(_p(n), h, _p(origin), _p(per), npart, _p(xp_), _p(rad),
                                      _p(u_), _p(Iu), _p(Ir), _p(alpha))
    if st != OK:
        raise OracleError(st)
    out = dict(Iu=Iu, Ir=Ir)
    if want_alpha:
        out["alpha"] = alpha
    return out


def cell_alpha(c0, h: float, R: float) -> float:
    """Level-set volume fraction of one cell (lowest corner c0 relative to the
    sphere centre)."""
    c = np.ascontiguousarray(c0, dtype=np.float64)
    return float(lib().ref_cell_alpha(_p(c), float(h), float(R)))


def grid_mean(case, f):
    n, _, _, _ = _grid(case)
    f_ = _f64(f)
    mean = np.zeros(3)
    st = lib().ref_grid_mean(_p(n), _p(f_), _p(mean))
    if st != OK:
        raise OracleError(st)
    return mean
