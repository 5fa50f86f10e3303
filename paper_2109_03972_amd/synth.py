"""Seeded synthetic inputs for the forcing loop and the pair pass.

This module only *draws* inputs: a collocated velocity field, sphere packings,
Lagrangian marker shells and rigid-body particle states.  It performs none of
the method's arithmetic (no delta kernel, no interpolation, no spreading, no
collision law); both the HIP path and the CPU oracle consume exactly the arrays
produced here.

Workloads (all in units h = 1, dt = 1) stand in for the paper's particle beds
(monodisperse fluidized bed, Sec. 3.5; bidisperse bed, Sec. 3.5) which have no
public dataset:

* ``single_sphere_64``: one sphere d = 16h in a 64^3 periodic box, 1 pass.
* ``suspension_128``: 200 spheres d = 12h in a 128^3 periodic box, 3 passes.
* ``bidisperse_bed_256x256x512``: 1000 d = 18h + 1000 d = 12h spheres at
  volume fraction 0.3 in a bottom slab, periodic x/y, walls in z, 5 passes.
* ``gradient_suspension_128``: ``suspension_128`` plus a seeded loss vector.
* ``polydisperse_bed_512``: 20000 lognormal spheres (median 12h, sigma 0.35,
  clipped to [8h, 24h]) at volume fraction 0.25 in a bottom slab of a 512^3
  grid, periodic x/y, walls in z, 5 passes.

Every quantity has its own stream spawned from ``SeedSequence(seed)`` so that
changing one recipe does not shift the others.

Marker shells: the marker count per sphere follows the shell volume of
thickness h divided by h^3 (Sec. 2.1 defines N_l dV_l as that shell volume),
rounded to the nearest integer, and each marker carries the volume
dV_l = shell / N_l.  Markers sit on the sphere surface at the points of the
generalized spiral of Saff & Kuijlaars (Math. Intelligencer 19, 1997), turned
by a seeded uniform random rotation per particle.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Case", "CONFIG_NAMES", "make_case", "spiral_points", "n_markers",
    "marker_volume", "fourier_field", "pack_spheres", "small_case",
    "default_params",
]

CONFIG_NAMES = (
    "single_sphere_64",
    "suspension_128",
    "bidisperse_bed_256x256x512",
    "gradient_suspension_128",
    "polydisperse_bed_512",
)

_MASTER_SEEDS = {name: 1001 + i for i, name in enumerate(CONFIG_NAMES)}

# stream indices spawned from the master seed
_S_FIELD, _S_SIZES, _S_POS, _S_VEL, _S_ROT, _S_CONTACT, _S_DISABLE, _S_LOSS = range(8)


def default_params() -> Dict[str, float]:
    """Physical and numerical parameters in units h = dt = 1.

    nu_f follows the paper's bed (nu dt / h^2 = 0.0247, Sec. 3.5); e_dry,
    mu_s, mu_k and zeta_min = 3e-3 r_p follow Sec. 3.4-3.5; eps_sep = 1.5h and
    C = 5.5 are the three-point values (Secs. 2.2.5-2.2.6); T_c = 10 dt (Sec. 2.2.7).
    ``c`` is 2 alpha_k dt with the first low-storage RK3 coefficient 4/15.
    St_crit = 5 and the k_n,grav constant 1e-3 follow Sec. 2.2.7; gravity is
    a small downward acceleration in these units.
    """
    return dict(
        kernel=3, n_iter=1, c=8.0 / 15.0, rho_f=1.0, nu_f=0.025,
        eps_sep=1.5, lub_C=5.5, zeta_min_factor=3e-3, e_dry=0.97, T_c=10.0,
        mu_s=0.11, mu_k=0.8, nu_poi=0.3, dt=1.0, disable_mode=1,
        disable_seed=0, gap_cut=3.0, normal_model=0, St_crit=5.0,
        gravity=(0.0, 0.0, -1.0e-4), kn_grav_eps=1e-3, st_switch=0,
    )


@dataclasses.dataclass
class Case:
    name: str
    n: Tuple[int, int, int]            # (nx, ny, nz)
    h: float
    origin: Tuple[float, float, float]
    periodic: Tuple[int, int, int]
    xp: np.ndarray        # float64 [3, np] particle centres
    up: np.ndarray        # float64 [3, np] translational velocities
    wp: np.ndarray        # float64 [3, np] angular velocities
    radius: np.ndarray    # float64 [np]
    mass: np.ndarray      # float64 [np]
    moff: np.ndarray      # int32 [np + 1] marker CSR offsets
    body: np.ndarray      # float64 [3, nm] marker offsets X_l - x_p
    dV: np.ndarray        # float64 [np] marker volume of each particle
    u0: Optional[np.ndarray]  # float64 [3, nz, ny, nx] or None (lazy)
    params: Dict[str, float]
    loss_b: Optional[np.ndarray] = None   # float64 [3, np] (gradient case)
    field_modes: Optional[dict] = None     # recipe of u0 (to regenerate)

    @property
    def np_(self) -> int:
        return int(self.xp.shape[1])

    @property
    def nm(self) -> int:
        return int(self.body.shape[1])

    @property
    def nodes(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def L(self) -> Tuple[float, float, float]:
        return tuple(self.n[a] * self.h for a in range(3))

    def field(self, device="cpu", dtype=None):
        """(Re)generate u0 from its recipe as a torch tensor (plumbing only)."""
        import torch
        return fourier_field_torch(self.n, self.h, self.origin, self.field_modes,
                                   device=device, dtype=dtype or torch.float64)


# ----------------------------------------------------------------------------
# marker shells
# ----------------------------------------------------------------------------

def n_markers(d: float, h: float = 1.0) -> int:
    """Marker count: shell volume pi h (3 d^2 + h^2) / 3 over h^3, rounded."""
    return int(math.floor(math.pi / 3.0 * (3.0 * (d / h) ** 2 + 1.0) + 0.5))


def marker_volume(d: float, h: float, nl: int) -> float:
    """dV_l of one marker: the thickness-h shell volume shared by nl markers."""
    return math.pi * h * (3.0 * d * d + h * h) / 3.0 / nl


def spiral_points(N: int) -> np.ndarray:
    """Generalized spiral points on the unit sphere (Saff & Kuijlaars 1997).

    Returns [N, 3].  h_k = -1 + 2(k-1)/(N-1), theta_k = arccos(h_k),
    phi_k = phi_{k-1} + 3.6/sqrt(N) / sqrt(1 - h_k^2) (mod 2 pi), with
    phi_1 = phi_N = 0.
    """
    if N == 1:
        return np.array([[0.0, 0.0, 1.0]])
    k = np.arange(1, N + 1, dtype=np.float64)
    hk = -1.0 + 2.0 * (k - 1.0) / (N - 1.0)
    theta = np.arccos(np.clip(hk, -1.0, 1.0))
    phi = np.zeros(N)
    inc = np.zeros(N)
    inner = slice(1, N - 1)
    inc[inner] = 3.6 / math.sqrt(N) / np.sqrt(1.0 - hk[inner] ** 2)
    phi[inner] = np.cumsum(inc[inner])
    phi = np.mod(phi, 2.0 * math.pi)
    phi[-1] = 0.0
    st = np.sin(theta)
    return np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(theta)], axis=1)


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotations from normalised Gaussian quaternions, [n,3,3]."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def build_markers(diam: np.ndarray, h: float, rng_rot: np.random.Generator):
    """Marker CSR, body offsets [3, nm] and per-particle dV for spheres."""
    npart = diam.shape[0]
    counts = np.array([n_markers(d, h) for d in diam], dtype=np.int64)
    moff = np.zeros(npart + 1, dtype=np.int64)
    moff[1:] = np.cumsum(counts)
    nm = int(moff[-1])
    if nm >= 2 ** 31:
        raise ValueError("marker count exceeds int32")
    rots = random_rotations(rng_rot, npart)
    body = np.empty((3, nm), dtype=np.float64)
    cache: Dict[int, np.ndarray] = {}
    for p in range(npart):
        c = int(counts[p])
        if c not in cache:
            cache[c] = spiral_points(c)
        pts = cache[c] @ rots[p].T * (0.5 * diam[p])
        body[:, moff[p]:moff[p + 1]] = pts.T
    dV = np.array([marker_volume(diam[p], h, int(counts[p])) for p in range(npart)])
    return moff.astype(np.int32), body, dV


# ----------------------------------------------------------------------------
# velocity field: sum of random Fourier modes
# ----------------------------------------------------------------------------

def draw_modes(rng: np.random.Generator, nmodes: int = 8, kmax: int = 4) -> dict:
    """8 modes, integer wavevectors with components in [-kmax, kmax] (k != 0),
    amplitude vectors ~ N(0, 1), phases ~ U[0, 2 pi)."""
    ks = []
    while len(ks) < nmodes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k)
    amp = rng.standard_normal((nmodes, 3))
    phase = rng.uniform(0.0, 2.0 * math.pi, size=nmodes)
    return dict(k=np.array(ks, dtype=np.int64), amp=amp, phase=phase)


def fourier_field_torch(n, h, origin, modes, device="cpu", dtype=None):
    """u(x) = sum_m a_m cos(2 pi k_m . (x / L) + theta_m) at the cell-centred
    nodes x = origin + (idx + 1/2) h, as a [3, nz, ny, nx] tensor."""
    import torch
    dtype = dtype or torch.float64
    nx, ny, nz = n
    L = [n[a] * h for a in range(3)]
    f64 = torch.float64
    coords = [((torch.arange(n[a], dtype=f64, device=device) + 0.5) * h + origin[a]) / L[a]
              for a in range(3)]
    out = torch.zeros((3, nz, ny, nx), dtype=f64, device=device)
    tmp = torch.empty((nz, ny, nx), dtype=f64, device=device)
    for m in range(modes["k"].shape[0]):
        kx, ky, kz = (int(v) for v in modes["k"][m])
        ax = 2.0 * math.pi * kx * coords[0] + float(modes["phase"][m])
        bc = (2.0 * math.pi * kz * coords[2])[:, None] + (2.0 * math.pi * ky * coords[1])[None, :]
        cbc, sbc = torch.cos(bc), torch.sin(bc)
        ca, sa = torch.cos(ax), torch.sin(ax)
        # cos(A + BC) = cos A cos BC - sin A sin BC
        torch.mul(cbc[:, :, None], ca[None, None, :], out=tmp)
        tmp.sub_(sbc[:, :, None] * sa[None, None, :])
        for c in range(3):
            out[c].add_(tmp, alpha=float(modes["amp"][m, c]))
    return out.to(dtype)


def fourier_field(n, h, origin, modes) -> np.ndarray:
    return fourier_field_torch(n, h, origin, modes).numpy()


# ----------------------------------------------------------------------------
# sphere packing (random sequential addition)
# ----------------------------------------------------------------------------

def pack_spheres(rng: np.random.Generator, L: Sequence[float], periodic: Sequence[int],
                 diam: np.ndarray, zlim: Tuple[float, float], min_gap: float = 0.0,
                 max_tries: int = 200000) -> np.ndarray:
    """Random sequential addition of spheres in the order given.

    Centres lie in [0, L) on the periodic axes; along z the whole sphere stays
    inside ``zlim``.  Any two spheres keep a surface gap >= ``min_gap`` under
    the minimum image.  Returns float64 [3, np].
    """
    L = np.asarray(L, dtype=np.float64)
    npart = diam.shape[0]
    R = 0.5 * diam
    cell = float(diam.max() + max(min_gap, 0.0))
    ncell = np.maximum(1, np.floor(L / cell).astype(np.int64))
    csize = L / ncell
    buckets: Dict[Tuple[int, int, int], List[int]] = {}
    pos = np.zeros((npart, 3))
    per = np.asarray(periodic, dtype=bool)
    for i in range(npart):
        lo = np.array([0.0, 0.0, zlim[0] + R[i]])
        hi = np.array([L[0], L[1], zlim[1] - R[i]])
        for a in range(3):
            if per[a]:
                lo[a], hi[a] = 0.0, L[a]
            elif a < 2:
                lo[a], hi[a] = R[i], L[a] - R[i]
        if hi[2] < lo[2]:
            raise ValueError("slab too thin for sphere")
        placed = False
        for _ in range(max_tries):
            c = lo + (hi - lo) * rng.random(3)
            ci = np.minimum((c / csize).astype(np.int64), ncell - 1)
            cand = []
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        key = [ci[0] + dx, ci[1] + dy, ci[2] + dz]
                        ok = True
                        for a in range(3):
                            if per[a]:
                                key[a] %= ncell[a]
                            elif key[a] < 0 or key[a] >= ncell[a]:
                                ok = False
                        if ok:
                            cand.extend(buckets.get(tuple(key), ()))
            if cand:
                idx = np.unique(np.asarray(cand))
                dxv = pos[idx] - c
                for a in range(3):
                    if per[a]:
                        dxv[:, a] -= L[a] * np.round(dxv[:, a] / L[a])
                dist = np.sqrt((dxv * dxv).sum(axis=1))
                if np.any(dist - R[idx] - R[i] < min_gap):
                    continue
            pos[i] = c
            buckets.setdefault(tuple(int(v) for v in ci), []).append(i)
            placed = True
            break
        if not placed:
            raise RuntimeError(f"packing failed at sphere {i}")
    return pos.T.copy()


def _exercise_contacts(rng, xp, radius, L, periodic, zlim, frac, depth=0.05):
    """Move a seeded fraction of particles into slight overlap (gap in
    [-depth, 0)) with their nearest neighbour so that contact branches run.
    A move is kept only if it creates no other overlap and keeps the sphere
    inside the slab."""
    npart = xp.shape[1]
    pos = xp.T.copy()
    per = np.asarray(periodic, dtype=bool)
    L = np.asarray(L)
    nmove = int(round(frac * npart))
    order = rng.permutation(npart)[: max(nmove * 3, nmove)]
    moved = 0
    for i in order:
        if moved >= nmove:
            break
        d = pos - pos[i]
        for a in range(3):
            if per[a]:
                d[:, a] -= L[a] * np.round(d[:, a] / L[a])
        dist = np.sqrt((d * d).sum(axis=1))
        gap = dist - radius - radius[i]
        gap[i] = np.inf
        j = int(np.argmin(gap))
        zeta = -depth * rng.random() - 1e-9 * depth
        nvec = -d[j] / dist[j]          # unit vector from j towards i
        # j's image nearest to i sits at pos[i] + d[j]; slide i along nvec
        newc = pos[i] + d[j] + nvec * (radius[i] + radius[j] + zeta)
        if newc[2] - radius[i] < zlim[0] or newc[2] + radius[i] > zlim[1]:
            continue
        if any((not per[a]) and (newc[a] - radius[i] < 0.0 or newc[a] + radius[i] > L[a])
               for a in range(2)):
            continue
        for a in range(3):
            if per[a]:
                newc[a] = newc[a] % L[a]
        d2 = pos - newc
        for a in range(3):
            if per[a]:
                d2[:, a] -= L[a] * np.round(d2[:, a] / L[a])
        g2 = np.sqrt((d2 * d2).sum(axis=1)) - radius - radius[i]
        g2[i] = np.inf
        g2[j] = np.inf
        if np.any(g2 < 0.0):
            continue
        pos[i] = newc
        moved += 1
    return pos.T.copy(), moved


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def _finish(name, n, periodic, xp, diam, rngs, n_iter, disable_mode, rho_p=1.3,
            loss=False, lazy_field=False):
    h = 1.0
    origin = (0.0, 0.0, 0.0)
    npart = xp.shape[1]
    radius = 0.5 * diam
    mass = rho_p * math.pi / 6.0 * diam ** 3
    up = rngs[_S_VEL].normal(0.0, 0.1, size=(3, npart))
    wp = rngs[_S_VEL].normal(0.0, 0.05, size=(3, npart))
    moff, body, dV = build_markers(diam, h, rngs[_S_ROT])
    modes = draw_modes(rngs[_S_FIELD])
    u0 = None if lazy_field else fourier_field(n, h, origin, modes)
    params = default_params()
    params["n_iter"] = n_iter
    params["disable_mode"] = disable_mode
    params["disable_seed"] = int(rngs[_S_DISABLE].integers(0, 2 ** 63 - 1))
    params["gap_cut"] = 2.0 * params["eps_sep"] if disable_mode else params["eps_sep"]
    loss_b = rngs[_S_LOSS].standard_normal((3, npart)) if loss else None
    return Case(name=name, n=tuple(n), h=h, origin=origin, periodic=tuple(periodic),
                xp=np.ascontiguousarray(xp), up=up, wp=wp, radius=radius, mass=mass,
                moff=moff, body=body, dV=dV, u0=u0, params=params, loss_b=loss_b,
                field_modes=modes)


def make_case(name: str, seed: Optional[int] = None, lazy_field: bool = False) -> Case:
    """Build one of the five named workloads with its master seed."""
    if name not in _MASTER_SEEDS:
        raise KeyError(name)
    seed = _MASTER_SEEDS[name] if seed is None else seed
    rngs = [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(8)]
    if name == "single_sphere_64":
        n = (64, 64, 64)
        xp = (np.array([32.0, 32.0, 32.0]) + rngs[_S_POS].uniform(-0.5, 0.5, 3)).reshape(3, 1)
        return _finish(name, n, (1, 1, 1), xp, np.array([16.0]), rngs, 1, 0, lazy_field=lazy_field)
    if name in ("suspension_128", "gradient_suspension_128"):
        n = (128, 128, 128)
        diam = np.full(200, 12.0)
        xp = pack_spheres(rngs[_S_POS], (128.0,) * 3, (1, 1, 1), diam, (-1e9, 1e9), min_gap=0.5)
        return _finish(name, n, (1, 1, 1), xp, diam, rngs, 3, 1,
                       loss=(name == "gradient_suspension_128"), lazy_field=lazy_field)
    if name == "bidisperse_bed_256x256x512":
        n = (256, 256, 512)
        diam = np.concatenate([np.full(1000, 18.0), np.full(1000, 12.0)])
        vol = float(np.sum(math.pi / 6.0 * diam ** 3))
        H = vol / (0.3 * n[0] * n[1])
        xp = pack_spheres(rngs[_S_POS], (256.0, 256.0, 512.0), (1, 1, 0), diam, (0.0, H))
        xp, _ = _exercise_contacts(rngs[_S_CONTACT], xp, 0.5 * diam, (256.0, 256.0, 512.0),
                                   (1, 1, 0), (0.0, H), 0.02)
        return _finish(name, n, (1, 1, 0), xp, diam, rngs, 5, 1, lazy_field=lazy_field)
    if name == "polydisperse_bed_512":
        n = (512, 512, 512)
        d = np.exp(rngs[_S_SIZES].normal(math.log(12.0), 0.35, size=20000))
        diam = np.clip(d, 8.0, 24.0)
        diam = -np.sort(-diam)          # pack largest first
        vol = float(np.sum(math.pi / 6.0 * diam ** 3))
        H = vol / (0.25 * n[0] * n[1])
        xp = pack_spheres(rngs[_S_POS], (512.0,) * 3, (1, 1, 0), diam, (0.0, H))
        xp, _ = _exercise_contacts(rngs[_S_CONTACT], xp, 0.5 * diam, (512.0,) * 3,
                                   (1, 1, 0), (0.0, H), 0.02)
        return _finish(name, n, (1, 1, 0), xp, diam, rngs, 5, 1, lazy_field=lazy_field)
    raise KeyError(name)


def small_case(seed: int, n=(40, 36, 44), periodic=(1, 1, 0), diameters=(12.0, 9.0, 7.0, 10.0),
               n_iter: int = 3, disable_mode: int = 1, min_gap: float = 0.3,
               touch: float = 0.0) -> Case:
    """A small polydisperse case for parity tests: a grid that is not a
    multiple of any tile edge, several spheres of different sizes, optional
    walls in z.  ``touch`` > 0 moves that fraction of spheres into contact."""
    rngs = [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(8)]
    diam = np.asarray(diameters, dtype=np.float64)
    L = tuple(float(v) for v in n)
    zlim = (0.0, L[2]) if not periodic[2] else (-1e9, 1e9)
    if not periodic[2]:
        # keep every marker at least 1h from a wall when disabling is off
        zlim = (1.6, L[2] - 1.6) if disable_mode == 0 else (0.0, L[2])
    xp = pack_spheres(rngs[_S_POS], L, periodic, diam, zlim, min_gap=min_gap)
    if touch > 0:
        zz = zlim if not periodic[2] else (-1e9, 1e9)
        xp, _ = _exercise_contacts(rngs[_S_CONTACT], xp, 0.5 * diam, L, periodic, zz, touch)
    c = _finish(f"small_{seed}", n, periodic, xp, diam, rngs, n_iter, disable_mode)
    return c
