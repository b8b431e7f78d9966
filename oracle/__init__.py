"""FP64 CPU oracle for the arbitrary-positioned SPH buffer update -- TEST INFRASTRUCTURE.

This package is the checker, not the product.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it.  It wraps
``sphbuf_oracle.c`` (plain C, FP64, built without FMA contraction) through ctypes and
shares no code with the GPU library.

Semantics follow arXiv 2406.16786, Section 3 (frames: Eq. 2D_transformation and
Eqs. rotation_axis .. 3D_transformation; inflow: Algorithm 1; outflow: Algorithm 2;
bidirectional: Algorithm 3).  See ``sphbuf_oracle.c`` for the step-by-step
definition used.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sphbuf_oracle.c")
_LIB = os.path.join(_HERE, "libsphbuf_oracle.so")

OK, ERR_ARG, ERR_CAPACITY, ERR_CFL, ERR_NONFINITE = 0, 1, 4, 5, 6
INLET, OUTLET, BIDIR = 1, 2, 3
BC_NONE, BC_VELOCITY, BC_PRESSURE = 0, 1, 2
PROFILE_PLUG, PROFILE_PARABOLIC_Y, PROFILE_PARABOLIC_R = 0, 1, 2
MAX_BUFFERS = 15
MAX_CARRIED = 16


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction; OpenMP over the
    per-particle loops, whose arithmetic does not depend on it); returns the .so
    path."""
    cmd = [
        "gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
        "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _CBuffer(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("origin", ctypes.c_double * 3),
        ("rot", ctypes.c_double * 9),
        ("half", ctypes.c_double * 3),
        ("margin", ctypes.c_double),
    ]


class _CBc(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("u", ctypes.c_double),
        ("radius", ctypes.c_double),
        ("p_b", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("c0", ctypes.c_double),
    ]


class _CFields(ctypes.Structure):
    _fields_ = [("vel", ctypes.c_int32 * 3), ("rho", ctypes.c_int32)]


class _CState(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n_carried", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("capacity", ctypes.c_int64),
        ("next_id", ctypes.c_int64),
        ("pos", ctypes.c_void_p * 3),
        ("carried", ctypes.c_void_p * MAX_CARRIED),
        ("label", ctypes.c_void_p),
        ("id", ctypes.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_rotation_2d.argtypes = [ctypes.c_double, dp]
        L.orc_rodrigues.argtypes = [dp, ctypes.c_double, dp]
        L.orc_rotation_from_direction.argtypes = [dp, dp]
        L.orc_rotation_from_direction.restype = ctypes.c_int
        L.orc_local_coords.argtypes = [ctypes.c_int, ctypes.POINTER(_CBuffer), ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_recycle_literal.argtypes = [ctypes.c_int, ctypes.POINTER(_CBuffer), dp, dp]
        L.orc_identify.argtypes = [ctypes.POINTER(_CBuffer), ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(_CState), ctypes.c_void_p]
        L.orc_identify.restype = ctypes.c_int
        L.orc_update.argtypes = [ctypes.POINTER(_CBuffer), ctypes.c_int, ctypes.POINTER(_CState),
                                 ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                 ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]
        L.orc_update.restype = ctypes.c_int
        L.orc_update_bc.argtypes = [ctypes.POINTER(_CBuffer), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.POINTER(_CState), ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]
        L.orc_update_bc.restype = ctypes.c_int
        L.orc_apply_bc.argtypes = [ctypes.POINTER(_CBuffer), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.POINTER(_CState)]
        L.orc_apply_bc.restype = ctypes.c_int
        L.orc_rotate_buffer.argtypes = [ctypes.POINTER(_CBuffer), ctypes.c_int, ctypes.c_int, dp, dp,
                                        ctypes.c_void_p, ctypes.POINTER(_CState)]
        L.orc_rotate_buffer.restype = ctypes.c_int
        L.orc_cell_list.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]
        L.orc_cell_list.restype = ctypes.c_int
        L.orc_sparse_active.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]
        L.orc_sparse_active.restype = ctypes.c_int64
        L.orc_cell_list_sparse.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p,
                                           ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_cell_list_sparse.restype = ctypes.c_int
        L.orc_neighbor_count.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_void_p]
        L.orc_neighbor_count.restype = None
        L.orc_update_local.argtypes = [ctypes.POINTER(_CBuffer), ctypes.c_int, ctypes.POINTER(_CState),
                                       ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]
        L.orc_update_local.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ------------------------------------------------------------------ frames ---

def rotation_2d(theta: float) -> np.ndarray:
    """Eq. (2D_transformation) as a 3x3 global->local matrix."""
    q = np.zeros(9)
    lib().orc_rotation_2d(float(theta), _dptr(q))
    return q.reshape(3, 3)


def rodrigues(n: Sequence[float], theta: float) -> np.ndarray:
    """Eq. (rotation_matrix) exactly as printed: R = I + S sin(t) + S^2 (1 - cos(t))."""
    nn = np.ascontiguousarray(n, dtype=np.float64)
    r = np.zeros(9)
    lib().orc_rodrigues(_dptr(nn), float(theta), _dptr(r))
    return r.reshape(3, 3)


def rotation_from_direction(d: Sequence[float]) -> np.ndarray:
    """Global->local frame whose X' axis points along d (reading Q = R^T)."""
    dd = np.ascontiguousarray(d, dtype=np.float64)
    if dd.size == 2:
        dd = np.array([dd[0], dd[1], 0.0])
    q = np.zeros(9)
    st = lib().orc_rotation_from_direction(_dptr(dd), _dptr(q))
    if st != OK:
        raise ValueError("direction must be a finite non-zero vector")
    return q.reshape(3, 3)


# ----------------------------------------------------------------- buffers ---

@dataclass
class Buffer:
    """One in-/outlet: kind, origin O', global->local matrix Q, half-extents, margin."""
    kind: int
    origin: Sequence[float]
    rot: np.ndarray
    half: Sequence[float]
    margin: float

    def c(self) -> _CBuffer:
        b = _CBuffer()
        b.kind = int(self.kind)
        o = list(self.origin) + [0.0] * (3 - len(self.origin))
        h = list(self.half) + [0.0] * (3 - len(self.half))
        for i in range(3):
            b.origin[i] = float(o[i])
            b.half[i] = float(h[i])
        rr = np.asarray(self.rot, dtype=np.float64).reshape(9)
        for i in range(9):
            b.rot[i] = float(rr[i])
        b.margin = float(self.margin)
        return b


@dataclass
class BC:
    """Boundary condition of one buffer (Section 4): velocity profile or boundary pressure."""
    kind: int = BC_NONE
    profile: int = PROFILE_PLUG
    u: float = 0.0
    radius: float = 1.0
    p_b: float = 0.0
    rho0: float = 1.0
    c0: float = 1.0

    def c(self) -> _CBc:
        b = _CBc()
        b.kind, b.profile = int(self.kind), int(self.profile)
        b.u, b.radius, b.p_b, b.rho0, b.c0 = (float(self.u), float(self.radius), float(self.p_b),
                                              float(self.rho0), float(self.c0))
        return b


@dataclass
class Fields:
    """Carried-field indices of the velocity components and the density (-1: absent)."""
    vel: Sequence[int] = (-1, -1, -1)
    rho: int = -1

    def c(self) -> _CFields:
        f = _CFields()
        v = list(self.vel) + [-1] * (3 - len(self.vel))
        for i in range(3):
            f.vel[i] = int(v[i])
        f.rho = int(self.rho)
        return f


def _cbcs(bcs: Optional[Sequence[BC]], nb: int):
    if bcs is None:
        return None
    arr = (_CBc * max(1, nb))()
    for i, b in enumerate(bcs):
        arr[i] = b.c()
    return arr


def _cbufs(bufs: Sequence[Buffer]):
    arr = (_CBuffer * max(1, len(bufs)))()
    for i, b in enumerate(bufs):
        arr[i] = b.c()
    return arr


def local_coords(dim: int, buf: Buffer, x, y, z=None) -> np.ndarray:
    """FP64 r' = Q (r - O') of FP32 positions; returns an (n, 3) array."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    n = x.size
    zz = np.ascontiguousarray(z if z is not None else np.zeros(n), dtype=np.float32)
    out = np.zeros((3, n))
    cb = buf.c()
    lib().orc_local_coords(dim, ctypes.byref(cb), n, x.ctypes.data, y.ctypes.data, zz.ctypes.data,
                           out[0].ctypes.data, out[1].ctypes.data, out[2].ctypes.data)
    return out.T.copy()


def recycle_literal(dim: int, buf: Buffer, r: Sequence[float]) -> np.ndarray:
    """Literal inverse transform of the paper: Q^T (Q (r - O') - [a,0,0]) + O' (FP64)."""
    rr = np.zeros(3)
    rr[: len(r)] = r
    out = np.zeros(3)
    cb = buf.c()
    lib().orc_recycle_literal(dim, ctypes.byref(cb), _dptr(rr), _dptr(out))
    return out[:dim].copy()


# ------------------------------------------------------------------- state ---

@dataclass
class State:
    """Host particle arrays, all of length ``capacity``; ``n`` live entries."""
    dim: int
    pos: List[np.ndarray]
    carried: List[np.ndarray]
    label: np.ndarray
    id: np.ndarray
    n: int
    next_id: int
    _keep: list = field(default_factory=list, repr=False)

    @property
    def capacity(self) -> int:
        return int(self.label.shape[0])

    def copy(self) -> "State":
        return State(self.dim, [p.copy() for p in self.pos], [c.copy() for c in self.carried],
                     self.label.copy(), self.id.copy(), self.n, self.next_id)

    def c(self) -> _CState:
        for p in self.pos + self.carried:
            assert p.dtype == np.float32 and p.flags.c_contiguous and p.shape[0] == self.capacity
        assert self.label.dtype == np.int32 and self.id.dtype == np.int64
        assert len(self.pos) == self.dim and len(self.carried) <= MAX_CARRIED
        s = _CState()
        s.dim = self.dim
        s.n_carried = len(self.carried)
        s.n = int(self.n)
        s.capacity = self.capacity
        s.next_id = int(self.next_id)
        for i, p in enumerate(self.pos):
            s.pos[i] = p.ctypes.data
        for i, c in enumerate(self.carried):
            s.carried[i] = c.ctypes.data
        s.label = self.label.ctypes.data
        s.id = self.id.ctypes.data
        return s


@dataclass
class UpdateResult:
    status: int
    gen: np.ndarray
    dele: np.ndarray
    n_labelled: np.ndarray


def identify(bufs: Sequence[Buffer], st: State, which: int = -1):
    """Algorithm 1, identification; returns (status, n_labelled per buffer)."""
    cs = st.c()
    cb = _cbufs(bufs)
    nl = np.zeros(max(1, len(bufs)), dtype=np.int64)
    rc = lib().orc_identify(cb, len(bufs), int(which), ctypes.byref(cs), nl.ctypes.data)
    return rc, nl[: len(bufs)]


def update(bufs: Sequence[Buffer], st: State, bcs: Optional[Sequence[BC]] = None,
           fields: Optional[Fields] = None) -> UpdateResult:
    """One buffer update (Algorithms 1-3); mutates ``st`` in place unless it fails.
    With boundary conditions, a particle recycled at a pressure boundary takes the
    density of Eq. (postulate-density)."""
    cs = st.c()
    cb = _cbufs(bufs)
    cap = max(1, st.n)
    gen = np.zeros(cap, dtype=np.int64)
    dele = np.zeros(cap, dtype=np.int64)
    ng, nd = ctypes.c_int64(0), ctypes.c_int64(0)
    nl = np.zeros(max(1, len(bufs)), dtype=np.int64)
    cbc = _cbcs(bcs, len(bufs))
    cf = fields.c() if fields is not None else None
    rc = lib().orc_update_bc(cb, ctypes.cast(cbc, ctypes.c_void_p) if cbc is not None else None,
                             ctypes.cast(ctypes.pointer(cf), ctypes.c_void_p) if cf is not None else None,
                             len(bufs), ctypes.byref(cs), gen.ctypes.data, ctypes.byref(ng),
                             dele.ctypes.data, ctypes.byref(nd), nl.ctypes.data)
    if rc == OK:
        st.n = int(cs.n)
        st.next_id = int(cs.next_id)
        return UpdateResult(rc, gen[: ng.value].copy(), dele[: nd.value].copy(), nl[: len(bufs)].copy())
    return UpdateResult(rc, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(len(bufs), np.int64))


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's per-particle loops (n <= 0 leaves the setting);
    returns the number the next call uses."""
    return int(lib().orc_set_threads(int(n)))


def update_local(bufs: Sequence[Buffer], st: State, lo, inv_cs: float, dims, cell_start: np.ndarray,
                 cell_idx: np.ndarray, n_labelled_in: Sequence[int]) -> UpdateResult:
    """The update with candidates only from the cells of a cell list (from
    cell_list on the dense grid lo, inv_cs, dims) near each check region: the
    paper's method on the CPU, for the CPU baseline.  Same results as update()."""
    cs = st.c()
    cb = _cbufs(bufs)
    lo32, d = _grid_args(st.dim, lo, dims)
    cap = max(1, st.n)
    gen = np.zeros(cap, dtype=np.int64)
    dele = np.zeros(cap, dtype=np.int64)
    ng, nd = ctypes.c_int64(0), ctypes.c_int64(0)
    nl = np.zeros(max(1, len(bufs)), dtype=np.int64)
    nl_in = np.zeros(max(1, len(bufs)), dtype=np.int64)
    nl_in[: len(bufs)] = n_labelled_in
    cell_start = np.ascontiguousarray(cell_start, dtype=np.int32)
    cell_idx = np.ascontiguousarray(cell_idx, dtype=np.int32)
    rc = lib().orc_update_local(cb, len(bufs), ctypes.byref(cs), lo32.ctypes.data, float(np.float32(inv_cs)),
                                d.ctypes.data, cell_start.ctypes.data, cell_idx.ctypes.data, nl_in.ctypes.data,
                                gen.ctypes.data, ctypes.byref(ng), dele.ctypes.data, ctypes.byref(nd),
                                nl.ctypes.data)
    if rc == OK:
        st.n = int(cs.n)
        st.next_id = int(cs.next_id)
        return UpdateResult(rc, gen[: ng.value].copy(), dele[: nd.value].copy(), nl[: len(bufs)].copy())
    return UpdateResult(rc, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(len(bufs), np.int64))


def apply_bc(bufs: Sequence[Buffer], bcs: Sequence[BC], fields: Fields, st: State) -> int:
    """Velocity / pressure boundary conditions on the buffer particles (Section 4);
    returns the status (ERR_CFL if a buffer particle lies outside its check region)."""
    cs = st.c()
    cb = _cbufs(bufs)
    cbc = _cbcs(bcs, len(bufs))
    cf = fields.c()
    return lib().orc_apply_bc(cb, ctypes.cast(cbc, ctypes.c_void_p), ctypes.cast(ctypes.pointer(cf), ctypes.c_void_p),
                              len(bufs), ctypes.byref(cs))


def rotate_buffer(bufs: List[Buffer], which: int, center: Sequence[float], m, fields: Optional[Fields],
                  st: State) -> int:
    """Rigid rotation of buffer ``which`` (1-based) and its particles about ``center``
    (Section 5.3); updates ``bufs[which - 1]`` in place and returns the status."""
    cs = st.c()
    cb = _cbufs(bufs)
    c = np.zeros(3)
    c[: len(center)] = center
    mm = np.ascontiguousarray(m, dtype=np.float64).reshape(9)
    cf = fields.c() if fields is not None else None
    rc = lib().orc_rotate_buffer(cb, len(bufs), int(which), _dptr(c), _dptr(mm),
                                 ctypes.cast(ctypes.pointer(cf), ctypes.c_void_p) if cf is not None else None,
                                 ctypes.byref(cs))
    b = cb[which - 1]
    bufs[which - 1] = Buffer(bufs[which - 1].kind, tuple(b.origin[i] for i in range(3)),
                             np.array([b.rot[i] for i in range(9)]).reshape(3, 3), bufs[which - 1].half,
                             bufs[which - 1].margin)
    return rc


def cell_list(dim: int, lo, inv_cs: float, dims, x, y, z=None):
    """Stable counting-sort cell list (cell_start[C+1], cell_idx[n]); FP32 binning."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    n = x.size
    zz = np.ascontiguousarray(z if z is not None else np.zeros(n), dtype=np.float32)
    lo32 = np.zeros(3, np.float32)
    lo32[: len(lo)] = lo
    d = np.ones(3, np.int32)
    d[: len(dims)] = dims
    C = int(d[0]) * int(d[1]) * (int(d[2]) if dim == 3 else 1)
    start = np.zeros(C + 1, np.int32)
    idx = np.zeros(max(1, n), np.int32)
    rc = lib().orc_cell_list(dim, lo32.ctypes.data, float(np.float32(inv_cs)), d.ctypes.data, n, x.ctypes.data,
                             y.ctypes.data, zz.ctypes.data, start.ctypes.data, idx.ctypes.data)
    if rc != OK:
        raise ValueError("bad cell-list arguments")
    return start, idx[:n]


def _grid_args(dim, lo, dims):
    lo32 = np.zeros(3, np.float32)
    lo32[: len(lo)] = lo
    d = np.ones(3, np.int32)
    d[: len(dims)] = dims
    return lo32, d


def sparse_active(dim: int, lo, inv_cs: float, dims, blog2: int, margin: int, x, y, z=None) -> np.ndarray:
    """Active-brick mask of the brick-sparse grid (occupied bricks dilated by margin)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    zz = np.ascontiguousarray(z if z is not None else np.zeros(x.size), dtype=np.float32)
    lo32, d = _grid_args(dim, lo, dims)
    bd = [(int(d[a]) + (1 << blog2) - 1) >> blog2 if a < dim else 1 for a in range(3)]
    act = np.zeros(bd[0] * bd[1] * bd[2], np.uint8)
    na = lib().orc_sparse_active(dim, lo32.ctypes.data, float(np.float32(inv_cs)), d.ctypes.data, blog2, margin,
                                 x.size, x.ctypes.data, y.ctypes.data, zz.ctypes.data, act.ctypes.data)
    if na < 0:
        raise ValueError("bad sparse-grid arguments")
    return act


def cell_list_sparse(dim: int, lo, inv_cs: float, dims, blog2: int, active: np.ndarray, x, y, z=None):
    """Stable counting-sort cell list on the brick-sparse grid (overflow key last)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    n = x.size
    zz = np.ascontiguousarray(z if z is not None else np.zeros(n), dtype=np.float32)
    lo32, d = _grid_args(dim, lo, dims)
    active = np.ascontiguousarray(active, dtype=np.uint8)
    C = int(active.sum()) * (1 << (dim * blog2)) + 1
    start = np.zeros(C + 1, np.int32)
    idx = np.zeros(max(1, n), np.int32)
    rc = lib().orc_cell_list_sparse(dim, lo32.ctypes.data, float(np.float32(inv_cs)), d.ctypes.data, blog2,
                                    active.ctypes.data, n, x.ctypes.data, y.ctypes.data, zz.ctypes.data,
                                    start.ctypes.data, idx.ctypes.data)
    if rc != OK:
        raise ValueError("bad sparse-grid arguments")
    return start, idx[:n]


def neighbor_count(dim: int, x, y, z=None, radius: float = 1.0, query=None) -> np.ndarray:
    """Brute-force neighbour counts (int32) of the query particles (all if None):
    other particles with FP64 squared distance ((dx*dx + dy*dy) + dz*dz) < radius^2."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    n = x.size
    zz = np.ascontiguousarray(z if z is not None else np.zeros(n), dtype=np.float32)
    if query is None:
        q = None
        nq = n
    else:
        q = np.ascontiguousarray(query, dtype=np.int64)
        nq = q.size
    out = np.zeros(max(1, nq), np.int32)
    lib().orc_neighbor_count(dim, n, x.ctypes.data, y.ctypes.data, zz.ctypes.data, float(radius),
                             None if q is None else q.ctypes.data, nq, out.ctypes.data)
    return out[:nq]
