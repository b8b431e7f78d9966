"""Seeded synthetic inputs for the SPH in-/outlet buffer update.

This module only draws inputs: particle lattices, buffer placements and the
prescribed velocity fields that move particles between updates.  It holds none of
the buffer method's arithmetic (no local frames, no crossing tests, no cell
lists), so both the GPU library's tests and the FP64 oracle can consume its output.

Buffers are described by placement only -- origin, the unit X' direction (the
in-/outflow direction), the 2-D rotation angle where there is one, half-extents
and margin.  Turning a direction into a rotation matrix is the method's job; the
consumer does it.

The shapes stand in for the paper's cases (Sections 5 and 6), whose geometry is
only given in figures: a straight 2-D channel, a bent 2-D channel with rotated
in-/outlets, a 3-D pipe with tilted in-/outlet planes, a 3-D branching pipe
network with bidirectional buffers, and a batch of hub-and-spoke domains.
All noise comes from numpy's PCG64 with fixed seeds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

INLET, OUTLET, BIDIR = 1, 2, 3
RHO0 = 1000.0


@dataclass
class BufferSpec:
    kind: int
    origin: tuple                 # O' (global)
    direction: tuple              # unit X' axis (global); in 2-D also given by ``angle``
    half: tuple                   # (a/2, b/2, c/2)
    margin: float                 # check-region margin delta
    angle: Optional[float] = None  # 2-D only: anticlockwise angle of X' from the x axis


@dataclass
class Workload:
    name: str
    dim: int
    dp: float
    cell_size: float
    lo: tuple
    hi: tuple
    n: int
    capacity: int
    pos: List[np.ndarray]          # float32, length capacity
    carried: List[np.ndarray]      # float32 fields copied on duplication, length capacity
    carried_names: List[str]
    label: np.ndarray              # int32, length capacity
    id: np.ndarray                 # int64, length capacity
    buffers: List[BufferSpec]
    dt: float
    steps: int
    seed_noise: int
    velocity: Callable = field(repr=False, default=None)  # (xp, pos_list, step, noise) -> list
    noise_scale: float = 0.0


def _alloc(dim: int, n: int, capacity: int, pts: np.ndarray, dp: float):
    pos = []
    for c in range(dim):
        a = np.zeros(capacity, dtype=np.float32)
        a[:n] = pts[:, c].astype(np.float32)
        pos.append(a)
    names = ["vx", "vy", "vz"][:dim] + ["mass", "rho", "p"]
    carried = [np.zeros(capacity, dtype=np.float32) for _ in names]
    carried[dim][:n] = np.float32(RHO0 * dp ** dim)
    carried[dim + 1][:n] = np.float32(RHO0)
    label = np.zeros(capacity, dtype=np.int32)
    ids = np.full(capacity, -1, dtype=np.int64)
    ids[:n] = np.arange(n, dtype=np.int64)
    return pos, carried, names, label, ids


def _jitter(rng, n, dim, dp, amp=0.3):
    return rng.uniform(-amp * dp, amp * dp, size=(n, dim))


def _block_order(idx: np.ndarray, block: int = 3) -> np.ndarray:
    """Permutation that groups lattice sites into block^dim tiles (integer lattice
    indices only), the kind of spatial ordering a solver keeps its particles in."""
    keys = [idx[:, c] // block for c in range(idx.shape[1])][::-1] + \
           [idx[:, c] % block for c in range(idx.shape[1])][::-1]
    return np.lexsort(keys[::-1])


def _finish(pts_idx, pts, order):
    if order == "lattice":
        return pts
    if order == "blocked":
        return pts[_block_order(pts_idx)]
    raise ValueError(order)


# ------------------------------------------------------------------ C1 ---

def channel2d(seed: int = 1, capacity_extra: int = 512, order: str = "lattice") -> Workload:
    """2-D straight channel 2.0 x 0.4, dp = 0.02, about 2,000 particles; axis-aligned
    inlet and outlet with 4-layer buffers; u = (1 + 0.05 xi, 0); dt = 0.25 dp."""
    dp = 0.02
    cs = 2.6 * dp
    rng = np.random.Generator(np.random.PCG64(seed))
    ii, jj = np.meshgrid(np.arange(100), np.arange(20), indexing="xy")
    idx = np.stack([ii.ravel(), jj.ravel()], axis=1)
    pts = (idx + 0.5) * dp + _jitter(rng, idx.shape[0], 2, dp)
    pts = _finish(idx, pts, order)
    n = pts.shape[0]
    cap = n + capacity_extra
    pos, carried, names, label, ids = _alloc(2, n, cap, pts, dp)
    half = (2 * dp, 0.2, 0.0)
    bufs = [BufferSpec(INLET, (2 * dp, 0.2, 0.0), (1.0, 0.0, 0.0), half, cs, angle=0.0),
            BufferSpec(OUTLET, (2.0 - 2 * dp, 0.2, 0.0), (1.0, 0.0, 0.0), half, cs, angle=0.0)]

    def velocity(xp, p, step, noise):
        # noise: standard normal per slot, shape (n,)
        return [1.0 + 0.05 * noise[0], 0.0 * noise[0]]

    return Workload("channel2d", 2, dp, cs, (-2 * cs, -2 * cs, 0.0), (2.0 + 2 * cs, 0.4 + 2 * cs, 0.0),
                    n, cap, pos, carried, names, label, ids, bufs, 0.25 * dp, 200, 1000, velocity, 1.0)


# ------------------------------------------------------------------ C2 ---

class _BentChannel:
    """Centerline: straight leg A (1.8 m at +30 deg), a clockwise circular bend of
    radius 0.4 through 75 deg, straight leg B (1.8 m at -45 deg); width W = 0.2."""

    def __init__(self):
        self.W = 0.2
        a0 = math.radians(30.0)
        self.tA = np.array([math.cos(a0), math.sin(a0)])
        self.nA = np.array([-self.tA[1], self.tA[0]])          # left normal
        self.P0 = np.array([0.0, 0.0])
        self.P1 = self.P0 + 1.8 * self.tA
        self.Rb = 0.4
        right = np.array([self.tA[1], -self.tA[0]])
        self.C = self.P1 + self.Rb * right
        self.phi0 = math.atan2(self.P1[1] - self.C[1], self.P1[0] - self.C[0])  # 120 deg
        self.phi1 = self.phi0 - math.radians(75.0)                               # 45 deg
        self.P2 = self.C + self.Rb * np.array([math.cos(self.phi1), math.sin(self.phi1)])
        b0 = math.radians(-45.0)
        self.tB = np.array([math.cos(b0), math.sin(b0)])
        self.nB = np.array([-self.tB[1], self.tB[0]])
        self.P3 = self.P2 + 1.8 * self.tB

    def frame(self, xp, x, y):
        """Signed distance s to the centerline (positive to the left) and the unit
        tangent, from the nearest of the three pieces; also an 'inside' mask."""
        W = self.W
        # leg A
        rxA, ryA = x - self.P0[0], y - self.P0[1]
        tA = rxA * self.tA[0] + ryA * self.tA[1]
        sA = rxA * self.nA[0] + ryA * self.nA[1]
        okA = (tA >= 0) & (tA <= 1.8)
        # leg B
        rxB, ryB = x - self.P2[0], y - self.P2[1]
        tB = rxB * self.tB[0] + ryB * self.tB[1]
        sB = rxB * self.nB[0] + ryB * self.nB[1]
        okB = (tB >= 0) & (tB <= 1.8)
        # bend (clockwise, the centre lies on the right: left side is outward)
        rxC, ryC = x - self.C[0], y - self.C[1]
        rho = xp.sqrt(rxC * rxC + ryC * ryC)
        phi = xp.arctan2(ryC, rxC)
        sC = rho - self.Rb
        okC = (phi <= self.phi0) & (phi >= self.phi1)
        big = 1e9
        dA = xp.where(okA, xp.abs(sA), big + 0 * sA)
        dB = xp.where(okB, xp.abs(sB), big + 0 * sB)
        dC = xp.where(okC, xp.abs(sC), big + 0 * sC)
        s = xp.where(dA <= xp.minimum(dB, dC), sA, xp.where(dB <= dC, sB, sC))
        rhos = xp.where(rho > 0, rho, 1.0 + 0 * rho)
        # clockwise tangent on the bend: (sin phi, -cos phi)
        txC, tyC = ryC / rhos, -rxC / rhos
        tx = xp.where(dA <= xp.minimum(dB, dC), self.tA[0] + 0 * x, xp.where(dB <= dC, self.tB[0] + 0 * x, txC))
        ty = xp.where(dA <= xp.minimum(dB, dC), self.tA[1] + 0 * x, xp.where(dB <= dC, self.tB[1] + 0 * x, tyC))
        inside = xp.minimum(xp.minimum(dA, dB), dC) < W / 2
        return s, tx, ty, inside


def bent_channel2d(seed: int = 2, capacity_extra: int = 4096, order: str = "lattice") -> Workload:
    """2-D bent channel, inlet at +30 deg and outlet at -45 deg, dp = 0.002, about
    206k particles; Poiseuille profile plus 2 % noise; dt = 0.25 dp."""
    dp = 0.002
    cs = 2.6 * dp
    g = _BentChannel()
    rng = np.random.Generator(np.random.PCG64(seed))
    s = np.linspace(0.0, 1.0, 257)[:, None]
    phis = g.phi0 + (g.phi1 - g.phi0) * s[:, 0]
    centre = np.concatenate([g.P0 + s * 1.8 * g.tA,
                             g.C + g.Rb * np.stack([np.cos(phis), np.sin(phis)], axis=1),
                             g.P2 + s * 1.8 * g.tB])
    bl = centre.min(axis=0) - g.W / 2 - 4 * dp
    bh = centre.max(axis=0) + g.W / 2 + 4 * dp
    nx = int(math.ceil((bh[0] - bl[0]) / dp))
    ny = int(math.ceil((bh[1] - bl[1]) / dp))
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    idx = np.stack([ii.ravel(), jj.ravel()], axis=1)
    base = bl + (idx + 0.5) * dp
    _, _, _, inside = g.frame(np, base[:, 0], base[:, 1])
    idx = idx[inside]
    pts = bl + (idx + 0.5) * dp + _jitter(rng, idx.shape[0], 2, dp)
    pts = _finish(idx, pts, order)
    n = pts.shape[0]
    cap = n + capacity_extra
    pos, carried, names, label, ids = _alloc(2, n, cap, pts, dp)
    half = (2 * dp, g.W / 2, 0.0)
    oin = g.P0 + 2 * dp * g.tA
    oout = g.P3 - 2 * dp * g.tB
    bufs = [BufferSpec(INLET, (oin[0], oin[1], 0.0), (g.tA[0], g.tA[1], 0.0), half, cs, angle=math.radians(30.0)),
            BufferSpec(OUTLET, (oout[0], oout[1], 0.0), (g.tB[0], g.tB[1], 0.0), half, cs,
                       angle=math.radians(-45.0))]
    umax = 1.0

    def velocity(xp, p, step, noise):
        s, tx, ty, _ = g.frame(xp, p[0], p[1])
        prof = umax * xp.clip(1.0 - (2.0 * s / g.W) ** 2, 0.0, None)
        return [prof * tx + 0.02 * umax * noise[0], prof * ty + 0.02 * umax * noise[1]]

    lo = (bl[0] - 2 * cs, bl[1] - 2 * cs, 0.0)
    hi = (bh[0] + 2 * cs, bh[1] + 2 * cs, 0.0)
    return Workload("bent_channel2d", 2, dp, cs, lo, hi, n, cap, pos, carried, names, label, ids, bufs,
                    0.25 * dp, 1000, 2000, velocity, 1.0)


# ------------------------------------------------------------------ C3 ---

def _rx(deg):
    t = math.radians(deg)
    return np.array([[1, 0, 0], [0, math.cos(t), -math.sin(t)], [0, math.sin(t), math.cos(t)]])


def _ry(deg):
    t = math.radians(deg)
    return np.array([[math.cos(t), 0, math.sin(t)], [0, 1, 0], [-math.sin(t), 0, math.cos(t)]])


def pipe3d(seed: int = 3, dp: float = 0.001, capacity_extra: Optional[int] = None,
           order: str = "lattice", length: float = 1.0, radius: float = 0.05) -> Workload:
    """3-D circular pipe along +z (R = 0.05, L = 1.0, dp = 0.001: about 7.85 M
    particles).  The inlet plane through the origin is tilted 20 deg about x, the
    outlet plane through (0, 0, L) 35 deg about y; 4-layer buffers; parabolic
    velocity along z plus 2 % noise; dt = 0.25 dp.  ``dp``/``length``/``radius``
    scale it down for small cases."""
    R, L = radius, length
    cs = 2.6 * dp
    rng = np.random.Generator(np.random.PCG64(seed))
    d_in = _rx(20.0) @ np.array([0.0, 0.0, 1.0])
    d_out = _ry(35.0) @ np.array([0.0, 0.0, 1.0])
    zlo = -R * math.tan(math.radians(20.0)) - dp
    zhi = L + R * math.tan(math.radians(35.0)) + dp
    nxy = int(math.ceil(2 * R / dp))
    nz = int(math.ceil((zhi - zlo) / dp))
    o = np.array([-R, -R, zlo])
    pts_all, idx_all = [], []
    zchunk = max(1, nz // 16)
    ii, jj = np.meshgrid(np.arange(nxy), np.arange(nxy), indexing="xy")
    ii, jj = ii.ravel(), jj.ravel()
    xy = np.stack([o[0] + (ii + 0.5) * dp, o[1] + (jj + 0.5) * dp], axis=1)
    disk = (xy[:, 0] ** 2 + xy[:, 1] ** 2) < R * R
    ii, jj, xy = ii[disk], jj[disk], xy[disk]
    for k0 in range(0, nz, zchunk):
        ks = np.arange(k0, min(nz, k0 + zchunk))
        z = o[2] + (ks + 0.5) * dp
        X = np.repeat(xy[None, :, 0], ks.size, axis=0).ravel()
        Y = np.repeat(xy[None, :, 1], ks.size, axis=0).ravel()
        Z = np.repeat(z[:, None], xy.shape[0], axis=1).ravel()
        keep = (X * d_in[0] + Y * d_in[1] + Z * d_in[2] > 0) & \
               (X * d_out[0] + Y * d_out[1] + (Z - L) * d_out[2] < 0)
        pts_all.append(np.stack([X[keep], Y[keep], Z[keep]], axis=1))
        idx_all.append(np.stack([np.tile(ii, ks.size)[keep], np.tile(jj, ks.size)[keep],
                                 np.repeat(ks, ii.size)[keep]], axis=1))
    pts = np.concatenate(pts_all)
    idx = np.concatenate(idx_all)
    pts = pts + _jitter(rng, pts.shape[0], 3, dp)
    pts = _finish(idx, pts, order)
    n = pts.shape[0]
    cap = n + (capacity_extra if capacity_extra is not None else max(4096, n // 100))
    pos, carried, names, label, ids = _alloc(3, n, cap, pts, dp)
    hin = (2 * dp, R / math.cos(math.radians(20.0)) + 2 * dp, R / math.cos(math.radians(20.0)) + 2 * dp)
    hout = (2 * dp, R / math.cos(math.radians(35.0)) + 2 * dp, R / math.cos(math.radians(35.0)) + 2 * dp)
    oin = 2 * dp * d_in
    oout = np.array([0.0, 0.0, L]) - 2 * dp * d_out
    bufs = [BufferSpec(INLET, tuple(oin), tuple(d_in), hin, cs),
            BufferSpec(OUTLET, tuple(oout), tuple(d_out), hout, cs)]
    umax = 1.0

    def velocity(xp, p, step, noise):
        r2 = p[0] * p[0] + p[1] * p[1]
        prof = umax * xp.clip(1.0 - r2 / (R * R), 0.0, None)
        return [0.02 * umax * noise[0], 0.02 * umax * noise[1], prof + 0.02 * umax * noise[2]]

    m = 2 * cs + 2 * dp
    lo = (-R - m, -R - m, zlo - m - 2 * dp)
    hi = (R + m, R + m, zhi + m + 2 * dp)
    return Workload("pipe3d", 3, dp, cs, lo, hi, n, cap, pos, carried, names, label, ids, bufs,
                    0.25 * dp, 500, 3000, velocity, 1.0)


# ------------------------------------------------------------ sprinkler ---

def sprinkler2d(seed: int = 8, dp: float = 0.002, arm: float = 0.1, radius: float = 0.02,
                omega: float = 2.0, n_background: int = 0, capacity: int = 200_000) -> Workload:
    """2-D rotating sprinkler (stand-in for the lawn sprinkler of Section 5.3): a
    velocity inlet of half-width R = 0.02 (profile 2500 (0.02^2 - y'^2), i.e.
    u = 1 m/s on the axis) at the end of an arm of length ``arm`` from the pivot
    (0, 0), pointing radially outward and turning at omega = 2 rad/s.  The buffer
    starts filled with a jittered lattice (4 layers); ``n_background`` optional
    resting particles are scattered over the lawn.  Particles move with their own
    (carried) velocity; dt = 0.25 dp / u."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = 4 * dp
    ny = int(round(2 * radius / dp))
    ii, jj = np.meshgrid(np.arange(4), np.arange(ny), indexing="xy")
    idx = np.stack([ii.ravel(), jj.ravel()], axis=1)
    loc = np.stack([-a / 2 + (idx[:, 0] + 0.5) * dp, -radius + (idx[:, 1] + 0.5) * dp], axis=1)
    loc = loc + _jitter(rng, loc.shape[0], 2, dp, amp=0.2)
    pts = loc + np.array([arm, 0.0])
    extent = 0.6
    if n_background:
        # resting particles on a jittered lattice over the lawn, in lattice order,
        # clear of the circle the turning buffer sweeps
        h = 2 * extent / math.sqrt(n_background)
        m_ = int(2 * extent / h)
        gi, gj = np.meshgrid(np.arange(m_), np.arange(m_), indexing="xy")
        bg = np.stack([-extent + (gi.ravel() + 0.5) * h, -extent + (gj.ravel() + 0.5) * h], axis=1)
        bg = bg + rng.uniform(-0.3 * h, 0.3 * h, size=bg.shape)
        bg = bg[np.hypot(bg[:, 0], bg[:, 1]) > arm + 3 * a]
        pts = np.concatenate([pts, bg])
    n = pts.shape[0]
    pos, carried, names, label, ids = _alloc(2, n, capacity, pts, dp)
    cs = 2.6 * dp
    bufs = [BufferSpec(INLET, (arm, 0.0, 0.0), (1.0, 0.0, 0.0), (a / 2, radius, 0.0), cs, angle=0.0)]
    m = 2 * cs
    wl = Workload("sprinkler2d", 2, dp, cs, (-extent - m, -extent - m, 0.0), (extent + m, extent + m, 0.0),
                  n, capacity, pos, carried, names, label, ids, bufs, 0.25 * dp / 1.0, 400, 8000, None, 0.0)
    wl.omega = omega
    wl.bc_u, wl.bc_radius = 1.0, radius
    return wl


def rotation_z(theta: float) -> np.ndarray:
    """Anticlockwise turn by theta about the z axis (row-major 3x3)."""
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def advect_carried(wl: Workload, pos: Sequence[np.ndarray], carried: Sequence[np.ndarray], n: int) -> None:
    """x <- fl32(x + fl32(v dt)) with each particle's own carried velocity."""
    for c in range(wl.dim):
        du = (carried[c][:n].astype(np.float64) * wl.dt).astype(np.float32)
        pos[c][:n] = (pos[c][:n] + du).astype(np.float32)


# -------------------------------------------------------------- helpers ---

def noise_for_step(wl: Workload, step: int, n: int) -> np.ndarray:
    """Standard-normal noise, one row per velocity component, for one step."""
    rng = np.random.Generator(np.random.PCG64(wl.seed_noise + step))
    return rng.standard_normal(size=(wl.dim, n))


def advect_host(wl: Workload, pos: Sequence[np.ndarray], n: int, step: int) -> None:
    """x <- fl32(x + fl32(u dt)) for the first n particles, on the host."""
    p64 = [p[:n].astype(np.float64) for p in pos]
    u = wl.velocity(np, p64, step, noise_for_step(wl, step, n))
    for c in range(wl.dim):
        du = (np.asarray(u[c], dtype=np.float64) * wl.dt).astype(np.float32)
        pos[c][:n] = (pos[c][:n] + du).astype(np.float32)


def random_box_particles(seed: int, n: int, dim: int, lo, hi, capacity: Optional[int] = None,
                         n_carried: int = 3):
    """Uniform random FP32 particles in [lo, hi); for small property tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cap = capacity if capacity is not None else n + 64
    pos = []
    for c in range(dim):
        a = np.zeros(cap, dtype=np.float32)
        a[:n] = rng.uniform(lo[c], hi[c], size=n).astype(np.float32)
        pos.append(a)
    carried = []
    for _ in range(n_carried):
        a = np.zeros(cap, dtype=np.float32)
        a[:n] = rng.standard_normal(n).astype(np.float32)
        carried.append(a)
    label = np.zeros(cap, dtype=np.int32)
    ids = np.full(cap, -1, dtype=np.int64)
    ids[:n] = np.arange(n)
    return pos, carried, label, ids


def random_unit(rng, dim: int) -> np.ndarray:
    v = rng.standard_normal(dim)
    v = v / np.linalg.norm(v)
    if dim == 2:
        v = np.array([v[0], v[1], 0.0])
    return v


# ------------------------------------------------------------------ C4 ---

def _perp_basis(t):
    a = np.array([1.0, 0.0, 0.0]) if abs(t[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    u = np.cross(t, a)
    u /= np.linalg.norm(u)
    v = np.cross(t, u)
    return u, v


def _child_dir(parent, polar_deg, azim):
    u, v = _perp_basis(parent)
    th = math.radians(polar_deg)
    d = math.cos(th) * parent + math.sin(th) * (math.cos(azim) * u + math.sin(azim) * v)
    return d / np.linalg.norm(d)


class _Tree:
    """Trunk (R 0.05, L 0.8) along +z from the origin; two daughters (R 0.04, L 0.6)
    at its end; the second daughter splits into two granddaughters (R 0.03, L 0.5);
    all lengths scaled by 1.08.
    Branch polar angles U(25, 50) deg from the parent, azimuths random; spheres of
    the parent radius fill the junctions."""

    def __init__(self, seed):
        rng = np.random.Generator(np.random.PCG64(seed))
        segs = []
        t0 = np.array([0.0, 0.0, 1.0])
        f = 1.08  # lengths scaled so that dp = 0.001 gives about 16 M particles
        segs.append((np.zeros(3), t0, 0.8 * f, 0.05))
        j1 = segs[0][0] + 0.8 * f * t0
        phi = rng.uniform(0, 2 * math.pi)
        d1 = _child_dir(t0, rng.uniform(25, 50), phi)
        d2 = _child_dir(t0, rng.uniform(25, 50), phi + math.pi + rng.uniform(-0.5, 0.5))
        segs.append((j1, d1, 0.6 * f, 0.04))
        segs.append((j1, d2, 0.6 * f, 0.04))
        j2 = j1 + 0.6 * f * d2
        psi = rng.uniform(0, 2 * math.pi)
        g1 = _child_dir(d2, rng.uniform(25, 50), psi)
        g2 = _child_dir(d2, rng.uniform(25, 50), psi + math.pi + rng.uniform(-0.5, 0.5))
        segs.append((j2, g1, 0.5 * f, 0.03))
        segs.append((j2, g2, 0.5 * f, 0.03))
        self.segs = segs
        self.spheres = [(j1, 0.05), (j2, 0.04)]
        self.leaves = [1, 3, 4]

    def inside(self, P):
        """Membership in the union of the segments and junction spheres; also the
        segment a point belongs to (nearest axis among those containing it)."""
        n = P.shape[0]
        seg_of = np.full(n, -1, dtype=np.int64)
        best = np.full(n, np.inf)
        for s, (a, t, L, R) in enumerate(self.segs):
            rel = P - a
            u = rel @ t
            rho2 = np.einsum("ij,ij->i", rel, rel) - u * u
            ok = (u > 0) & (u < L) & (rho2 < R * R)
            better = ok & (rho2 < best)
            seg_of[better] = s
            best[better] = rho2[better]
        for (c, R), s_par in zip(self.spheres, (0, 2)):
            d2 = np.einsum("ij,ij->i", P - c, P - c)
            ok = (d2 < R * R) & (seg_of < 0)
            seg_of[ok] = s_par
        return seg_of >= 0, seg_of

    def frame(self, xp, x, y, z):
        """Segment axis direction and radial profile factor for the velocity."""
        best = None
        tx = ty = tz = prof = None
        for a, t, L, R in self.segs:
            rx, ry, rz = x - a[0], y - a[1], z - a[2]
            u = rx * t[0] + ry * t[1] + rz * t[2]
            uc = xp.clip(u, 0.0, L)
            dx, dy, dz = rx - uc * t[0], ry - uc * t[1], rz - uc * t[2]
            d2 = dx * dx + dy * dy + dz * dz
            rho2 = rx * rx + ry * ry + rz * rz - u * u
            pr = xp.clip(1.0 - rho2 / (R * R), 0.0, None)
            if best is None:
                best, tx, ty, tz, prof = d2, t[0] + 0 * x, t[1] + 0 * x, t[2] + 0 * x, pr
            else:
                take = d2 < best
                best = xp.where(take, d2, best)
                tx = xp.where(take, t[0] + 0 * x, tx)
                ty = xp.where(take, t[1] + 0 * x, ty)
                tz = xp.where(take, t[2] + 0 * x, tz)
                prof = xp.where(take, pr, prof)
        return tx, ty, tz, prof


def tree3d(seed: int = 4, dp: float = 0.001, capacity_extra: Optional[int] = None, order: str = "lattice") -> Workload:
    """3-D branching pipe network (trunk, two daughters, two granddaughters), about
    16 M particles at dp = 0.001; one bidirectional buffer at the trunk inlet and one
    at each of the three leaf outlets, X' pointing into the domain; reversing
    sinusoidal velocity (period 200 dt) with a parabolic profile per segment plus
    2 % noise, so every buffer both generates and deletes; dt = 0.25 dp."""
    tree = _Tree(seed)
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    idx_all = []
    # lattice sites ((i + 1/2) dp, ...) inside the union; each site is produced by
    # the pass of the segment that owns it.  Per z-slice only the bounding box of
    # the axis points within R of the slice is scanned.
    for s, (a, t, L, R) in enumerate(tree.segs):
        zlo = min(a[2], a[2] + L * t[2]) - R - dp
        zhi = max(a[2], a[2] + L * t[2]) + R + dp
        k0, k1 = int(math.floor(zlo / dp)), int(math.ceil(zhi / dp))
        for k in range(k0, k1):
            z = (k + 0.5) * dp
            if abs(t[2]) < 1e-9:
                if abs(a[2] - z) > R:
                    continue
                ua, ub = 0.0, L
            else:
                u1, u2 = (z - R - a[2]) / t[2], (z + R - a[2]) / t[2]
                ua, ub = max(0.0, min(u1, u2)), min(L, max(u1, u2))
                if ua > ub:
                    ua = ub = min(max(u1, 0.0), L)
            pa, pb = a + ua * t, a + ub * t
            x0 = int(math.floor((min(pa[0], pb[0]) - R) / dp)) - 1
            x1 = int(math.ceil((max(pa[0], pb[0]) + R) / dp)) + 1
            y0 = int(math.floor((min(pa[1], pb[1]) - R) / dp)) - 1
            y1 = int(math.ceil((max(pa[1], pb[1]) + R) / dp)) + 1
            I, J = np.meshgrid(np.arange(x0, x1), np.arange(y0, y1), indexing="ij")
            I, J = I.ravel(), J.ravel()
            P = np.stack([(I + 0.5) * dp, (J + 0.5) * dp, np.full(I.size, z)], axis=1)
            ins, seg = tree.inside(P)
            keep = ins & (seg == s)
            if keep.any():
                idx_all.append(np.stack([I[keep], J[keep], np.full(int(keep.sum()), k)], axis=1))
    idx = np.concatenate(idx_all)
    # global lattice order: z slowest, then y, then x
    idx = idx[np.lexsort((idx[:, 0], idx[:, 1], idx[:, 2]))]
    pts = (idx + 0.5) * dp + _jitter(rng, idx.shape[0], 3, dp)
    pts = _finish(idx, pts, order)
    n = pts.shape[0]
    cap = n + (capacity_extra if capacity_extra is not None else max(8192, n // 50))
    pos, carried, names, label, ids = _alloc(3, n, cap, pts, dp)
    bufs = []
    a, t, L, R = tree.segs[0]
    o = a + 2 * dp * t
    bufs.append(BufferSpec(BIDIR, tuple(o), tuple(t), (2 * dp, R + 2 * dp, R + 2 * dp), 2.6 * dp))
    for s in tree.leaves:
        a, t, L, R = tree.segs[s]
        e = a + L * t
        o = e - 2 * dp * t
        bufs.append(BufferSpec(BIDIR, tuple(o), tuple(-t), (2 * dp, R + 2 * dp, R + 2 * dp), 2.6 * dp))
    dt = 0.25 * dp
    period = 200

    def velocity(xp, p, step, noise):
        tx, ty, tz, prof = tree.frame(xp, p[0], p[1], p[2])
        amp = math.sin(2 * math.pi * step / period)
        return [amp * prof * tx + 0.02 * noise[0], amp * prof * ty + 0.02 * noise[1],
                amp * prof * tz + 0.02 * noise[2]]

    m = 2 * 2.6 * dp + 2 * dp
    lo = tuple(pts.min(axis=0) - m)
    hi = tuple(pts.max(axis=0) + m)
    wl = Workload("tree3d", 3, dp, 2.6 * dp, lo, hi, n, cap, pos, carried, names, label, ids, bufs,
                  dt, 500, 4000, velocity, 1.0)
    wl.tree = tree
    return wl


# ------------------------------------------------------------------ C5 ---

def _hub_lattice(dim, dp, Rh, legs, r, L):
    """Lattice sites ((i + 1/2) dp) in a hub disk/sphere of radius Rh at the origin
    united with straight legs (half-width / radius r) from the origin to distance L
    along the unit directions in legs; each site once."""
    def inside(P):
        ok = np.einsum("ij,ij->i", P, P) < Rh * Rh
        for t in legs:
            u = P @ t[: P.shape[1]]
            rho2 = np.einsum("ij,ij->i", P, P) - u * u
            ok |= (u > 0) & (u < L) & (rho2 < r * r)
        return ok
    out = []
    ext = L + r + 2 * dp
    n1 = int(math.ceil(ext / dp))
    if dim == 2:
        ax = np.arange(-n1, n1)
        for c in range(0, ax.size, 256):
            I, J = np.meshgrid(ax, ax[c:c + 256], indexing="ij")
            idx = np.stack([I.ravel(), J.ravel()], axis=1)
            P = (idx + 0.5) * dp
            # cheap reject: outside every leg's and the hub's bounding disc
            out.append(idx[inside(P)])
        return np.concatenate(out)
    # 3-D: per z-slice, the union's bounding box in x, y
    for k in range(-n1, n1):
        z = (k + 0.5) * dp
        boxes = []
        if abs(z) < Rh:
            boxes.append((-Rh, Rh, -Rh, Rh))
        for t in legs:
            if abs(t[2]) < 1e-9:
                if abs(z) > r:
                    continue
                ua, ub = 0.0, L
            else:
                u1, u2 = (z - r) / t[2], (z + r) / t[2]
                ua, ub = max(0.0, min(u1, u2)), min(L, max(u1, u2))
                if ua > ub:
                    continue
            pa, pb = ua * t, ub * t
            boxes.append((min(pa[0], pb[0]) - r, max(pa[0], pb[0]) + r, min(pa[1], pb[1]) - r, max(pa[1], pb[1]) + r))
        if not boxes:
            continue
        bx = np.array(boxes)
        x0, x1 = int(math.floor(bx[:, 0].min() / dp)) - 1, int(math.ceil(bx[:, 1].max() / dp)) + 1
        y0, y1 = int(math.floor(bx[:, 2].min() / dp)) - 1, int(math.ceil(bx[:, 3].max() / dp)) + 1
        I, J = np.meshgrid(np.arange(x0, x1), np.arange(y0, y1), indexing="ij")
        I, J = I.ravel(), J.ravel()
        P = np.stack([(I + 0.5) * dp, (J + 0.5) * dp, np.full(I.size, z)], axis=1)
        keep = inside(P)
        if keep.any():
            out.append(np.stack([I[keep], J[keep], np.full(int(keep.sum()), k)], axis=1))
    return np.concatenate(out)


def hub_domain(index: int, n_target: int, dim: int, n_legs: int, seed_base: int = 5000) -> Workload:
    """One hub-and-spoke domain: a hub of radius 1 with n_legs straight legs (radius
    0.35, reaching distance 4 from the centre) in random directions at least 40 deg
    apart; dp chosen so the domain holds about n_target particles.  Leg 0 ends in an
    inlet, the others in outlets; a single leg ends in a bidirectional buffer with
    oscillating flow.  Poiseuille flow along each leg, 2 % noise, dt = 0.25 dp."""
    rng = np.random.Generator(np.random.PCG64(seed_base + index))
    Rh, r, L = 1.0, 0.35, 4.0
    legs = []
    while len(legs) < n_legs:
        v = rng.standard_normal(3)
        if dim == 2:
            v[2] = 0.0
        v /= np.linalg.norm(v)
        if all(float(v @ w) < math.cos(math.radians(40.0)) for w in legs):
            legs.append(v)
    if dim == 2:
        vol = math.pi * Rh * Rh + n_legs * 2 * r * (L - Rh)
    else:
        vol = 4.0 / 3.0 * math.pi * Rh ** 3 + n_legs * math.pi * r * r * (L - Rh)
    dp = (vol / n_target) ** (1.0 / dim)
    idx = _hub_lattice(dim, dp, Rh, legs, r, L)
    idx = idx[np.lexsort(tuple(idx[:, c] for c in range(dim)))]
    pts = (idx + 0.5) * dp + _jitter(rng, idx.shape[0], dim, dp)
    n = pts.shape[0]
    cap = n + max(1024, n // 20)
    pos, carried, names, label, ids = _alloc(dim, n, cap, pts, dp)
    bufs = []
    for j, t in enumerate(legs):
        e = L * t
        o = e - 2 * dp * t
        half = (2 * dp, r + 2 * dp, r + 2 * dp if dim == 3 else 0.0)
        if n_legs == 1:
            kind, d = BIDIR, -t
        elif j == 0:
            kind, d = INLET, -t
        else:
            kind, d = OUTLET, t
        ang = math.atan2(d[1], d[0]) if dim == 2 else None
        bufs.append(BufferSpec(kind, tuple(o), tuple(d), half, 2.6 * dp, angle=ang))
    sign = np.array([-1.0 if (j == 0 or n_legs == 1) else 1.0 for j in range(n_legs)])

    def velocity(xp, p, step, noise):
        x, y = p[0], p[1]
        z = p[2] if dim == 3 else 0.0 * x
        amp = math.sin(2 * math.pi * step / 200.0) if n_legs == 1 else 1.0
        vx, vy, vz = 0.0 * x, 0.0 * x, 0.0 * x
        for j, t in enumerate(legs):
            u = x * t[0] + y * t[1] + z * t[2]
            rho2 = x * x + y * y + z * z - u * u
            prof = xp.clip(1.0 - rho2 / (r * r), 0.0, None) * ((u > Rh) & (u < L + r))
            s = amp * sign[j]
            vx = vx + s * prof * t[0]
            vy = vy + s * prof * t[1]
            vz = vz + s * prof * t[2]
        u_ = [vx + 0.02 * noise[0], vy + 0.02 * noise[1]]
        if dim == 3:
            u_.append(vz + 0.02 * noise[2])
        return u_

    m = 2 * 2.6 * dp + 2 * dp
    lo = tuple(list(pts.min(axis=0) - m) + [0.0] * (3 - dim))
    hi = tuple(list(pts.max(axis=0) + m) + [0.0] * (3 - dim))
    wl = Workload(f"hub{index}", dim, dp, 2.6 * dp, lo, hi, n, cap, pos, carried, names, label, ids, bufs,
                  0.25 * dp, 200, 6000 + 100 * index, velocity, 1.0)
    return wl


def hub_batch(n_domains: int = 64, n_min: float = 1e4, n_max: float = 2e6, seed: int = 5) -> List[Workload]:
    """A batch of independent hub-and-spoke domains: dimension 2 or 3 with equal
    odds, particle counts log-uniform over [n_min, n_max], 1-6 legs each."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_domains):
        dim = int(rng.integers(2, 4))
        n_t = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        n_legs = int(rng.integers(1, 7))
        out.append(hub_domain(i, n_t, dim, n_legs))
    return out
