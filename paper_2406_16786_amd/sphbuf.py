"""ctypes binding of ``libsphbuf.so`` (declared in ``include/sphbuf.h``).

Argument marshalling only: every function keeps the C name and forwards to the
library, which runs every step of the buffer update in its own HIP kernels.
PyTorch supplies device memory (``tensor.data_ptr()``) and the stream.  There is
no fallback: if the shared library is missing, loading it raises.

Contexts and batches still alive when the interpreter exits are destroyed by an
``atexit`` hook (batches first, then contexts), while the HIP runtime is still
up: left to garbage collection at interpreter teardown, their HIP calls could
run after the runtime (or a profiler attached to it) has shut down.
"""
from __future__ import annotations

import atexit
import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsphbuf.so")

SPH_OK, SPH_ERR_ARG, SPH_ERR_ROTATION, SPH_ERR_OVERLAP, SPH_ERR_CAPACITY = 0, 1, 2, 3, 4
SPH_ERR_CFL, SPH_ERR_NONFINITE, SPH_ERR_TOO_MANY_BUFFERS, SPH_ERR_EVENTS = 5, 6, 7, 8
SPH_ERR_HIP, SPH_ERR_STATE = 9, 10
SPH_INLET, SPH_OUTLET, SPH_BIDIR = 1, 2, 3
SPH_MAX_BUFFERS = 15
SPH_MAX_CARRIED = 16
SPH_MAX_EVENTS_LIMIT = 4096
SPH_UPDATE_MERGED, SPH_UPDATE_CELLS = 0, 1
UPDATE_PATHS = {"merged": SPH_UPDATE_MERGED, "cells": SPH_UPDATE_CELLS}
SPH_BUILD_AUTO, SPH_BUILD_COUNTING, SPH_BUILD_BUCKETED = 0, 1, 2
BUILD_METHODS = {"auto": SPH_BUILD_AUTO, "counting": SPH_BUILD_COUNTING, "bucketed": SPH_BUILD_BUCKETED}
SPH_STATE_BLOB_BYTES = 136

EXPORTED = (
    "sph_create", "sph_destroy", "sph_buffer_define", "sph_celllist_build", "sph_buffer_identify",
    "sph_buffer_update", "sph_buffer_update_async", "sph_buffer_update_fullscan",
    "sph_buffer_update_fullscan_async", "sph_last_result", "sph_last_events", "sph_celllist_view",
    "sph_build_stats", "sph_build_retune",
    "sph_state_get", "sph_state_set", "sph_rotation_2d", "sph_rotation_axis_angle",
    "sph_rotation_from_direction", "sph_check_rotation", "sph_grid_cover", "sph_guard_band",
    "sph_status_str", "sph_profile_enable", "sph_profile_read", "sph_grid_fit",
    "sph_batch_create", "sph_batch_destroy", "sph_batch_set_mode", "sph_batch_set_count_block",
    "sph_batch_set_gather", "sph_batch_get_config",
    "sph_batch_step", "sph_batch_results", "sph_batch_tune",
    "sph_set_fields", "sph_buffer_set_bc", "sph_buffer_apply_bc", "sph_buffer_rotate", "sph_neighbor_count",
    "sph_state_export", "sph_state_import", "sph_batch_graph_capture", "sph_batch_graph_launch",
    "sph_batch_profile_enable", "sph_batch_profile_read",
    "sph_buffer_rotate_async", "sph_buffer_apply_bc_async", "sph_last_bc_status", "sph_buffer_cover",
    "sph_celllist_build_noalloc",
)
SPH_NOALLOC_MAX_PARTICLES = 1 << 20
SPH_NOALLOC_MAX_CELLS = 1 << 20
BATCH_PHASES = ("count", "scan", "scatter", "classify", "finalize")
SPH_BATCH_KERNELS, SPH_BATCH_GRAPH = 0, 1
SPH_NPHASE = 12
PHASES = ("count", "scan", "scatter", "classify", "fullscan", "finalize", "bc", "rotate", "candidates", "neighbor",
          "cover", "sort")
SPH_BC_NONE, SPH_BC_VELOCITY, SPH_BC_PRESSURE = 0, 1, 2
SPH_PROFILE_PLUG, SPH_PROFILE_PARABOLIC_Y, SPH_PROFILE_PARABOLIC_R = 0, 1, 2


class sph_particles(ctypes.Structure):
    _fields_ = [
        ("pos", ctypes.c_void_p * 3),
        ("carried", ctypes.c_void_p * SPH_MAX_CARRIED),
        ("n_carried", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("label", ctypes.c_void_p),
        ("id", ctypes.c_void_p),
        ("n_dev", ctypes.c_void_p),
        ("capacity", ctypes.c_int64),
    ]


class sph_config(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("cell_size", ctypes.c_double),
        ("dp", ctypes.c_double),
        ("capacity", ctypes.c_int64),
        ("max_events", ctypes.c_int64),
        ("next_id", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("brick_log2", ctypes.c_int32),
        ("brick_margin", ctypes.c_int32),
        ("update_path", ctypes.c_int32),
        ("build_method", ctypes.c_int32),
    ]


class sph_result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("n_buffers", ctypes.c_int32),
        ("n_generated", ctypes.c_int64),
        ("n_deleted", ctypes.c_int64),
        ("n_before", ctypes.c_int64),
        ("n_after", ctypes.c_int64),
        ("next_id", ctypes.c_int64),
        ("n_labelled", ctypes.c_int64 * SPH_MAX_BUFFERS),
    ]


class sph_fields(ctypes.Structure):
    _fields_ = [("vel", ctypes.c_int32 * 3), ("rho", ctypes.c_int32)]


class sph_bc(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("u", ctypes.c_double),
        ("radius", ctypes.c_double),
        ("p_b", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("c0", ctypes.c_double),
    ]


class SphError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = int(status)
        super().__init__(f"{what}: {sph_status_str(status)} (status {status})")


_lib = None
_live_ctx: set = set()
_live_batch: set = set()


@atexit.register
def _destroy_live_handles() -> None:
    """Destroy what the program left alive, batches before their member contexts."""
    if _lib is None:
        return
    for b in list(_live_batch):
        _live_batch.discard(b)
        _lib.sph_batch_destroy(b)
    for c in list(_live_ctx):
        _live_ctx.discard(c)
        _lib.sph_destroy(c)


_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)
_VP = ctypes.c_void_p


def lib() -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "sph_create": ([ctypes.POINTER(sph_config), ctypes.POINTER(_VP)], ctypes.c_int),
            "sph_destroy": ([_VP], ctypes.c_int),
            "sph_buffer_define": ([_VP, ctypes.c_int, _D, _D, _D, ctypes.c_double, _I32], ctypes.c_int),
            "sph_celllist_build": ([_VP, ctypes.POINTER(sph_particles)], ctypes.c_int),
            "sph_grid_fit": ([_VP, ctypes.POINTER(sph_particles)], ctypes.c_int),
            "sph_buffer_identify": ([_VP, ctypes.POINTER(sph_particles), ctypes.c_int32], ctypes.c_int),
            "sph_buffer_update": ([_VP, ctypes.POINTER(sph_particles), _I64, _I64], ctypes.c_int),
            "sph_buffer_update_async": ([_VP, ctypes.POINTER(sph_particles)], ctypes.c_int),
            "sph_buffer_update_fullscan": ([_VP, ctypes.POINTER(sph_particles), _I64, _I64], ctypes.c_int),
            "sph_buffer_update_fullscan_async": ([_VP, ctypes.POINTER(sph_particles)], ctypes.c_int),
            "sph_last_result": ([_VP, ctypes.POINTER(sph_result)], ctypes.c_int),
            "sph_last_events": ([_VP, _I64, _I64, ctypes.c_int64, _I64, _I64], ctypes.c_int),
            "sph_celllist_view": ([_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP), _I64, _I32], ctypes.c_int),
            "sph_build_stats": ([_VP, _I32, ctypes.POINTER(ctypes.c_double), _I64], ctypes.c_int),
            "sph_build_retune": ([_VP], ctypes.c_int),
            "sph_state_get": ([_VP, _I64, _I64], ctypes.c_int),
            "sph_state_set": ([_VP, ctypes.c_int64, _I64], ctypes.c_int),
            "sph_state_export": ([_VP, _VP, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
            "sph_state_import": ([_VP, _VP, ctypes.c_size_t], ctypes.c_int),
            "sph_batch_graph_capture": ([_VP], ctypes.c_int),
            "sph_batch_graph_launch": ([_VP], ctypes.c_int),
            "sph_batch_profile_enable": ([_VP, ctypes.c_int32], ctypes.c_int),
            "sph_batch_profile_read": ([_VP, _D, _I64, ctypes.c_int32], ctypes.c_int),
            "sph_rotation_2d": ([ctypes.c_double, _D], ctypes.c_int),
            "sph_rotation_axis_angle": ([_D, ctypes.c_double, _D], ctypes.c_int),
            "sph_rotation_from_direction": ([_D, _D], ctypes.c_int),
            "sph_check_rotation": ([ctypes.c_int32, _D], ctypes.c_int),
            "sph_grid_cover": ([ctypes.c_int32, _D, ctypes.c_double, _I32, _D, _D, _D, ctypes.c_double, _I32, _I32,
                                ctypes.c_int64, _I64], ctypes.c_int),
            "sph_guard_band": ([ctypes.c_int32, _D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double],
                               ctypes.c_double),
            "sph_status_str": ([ctypes.c_int], ctypes.c_char_p),
            "sph_profile_enable": ([_VP, ctypes.c_int32], ctypes.c_int),
            "sph_set_fields": ([_VP, ctypes.POINTER(sph_fields)], ctypes.c_int),
            "sph_buffer_set_bc": ([_VP, ctypes.c_int32, ctypes.POINTER(sph_bc)], ctypes.c_int),
            "sph_buffer_apply_bc": ([_VP, ctypes.POINTER(sph_particles)], ctypes.c_int),
            "sph_buffer_rotate": ([_VP, ctypes.POINTER(sph_particles), ctypes.c_int32, _D, _D], ctypes.c_int),
            "sph_buffer_rotate_async": ([_VP, ctypes.POINTER(sph_particles), ctypes.c_int32, _D, _D], ctypes.c_int),
            "sph_buffer_apply_bc_async": ([_VP, ctypes.POINTER(sph_particles)], ctypes.c_int),
            "sph_last_bc_status": ([_VP], ctypes.c_int),
            "sph_buffer_cover": ([_VP, ctypes.c_int32, _I32, _I32, ctypes.c_int64, _I64], ctypes.c_int),
            "sph_celllist_build_noalloc": ([ctypes.c_int32, _D, ctypes.c_double, _I32, _VP, _VP, _VP, _VP,
                                            ctypes.c_int64, _VP, _VP, _VP], ctypes.c_int),
            "sph_neighbor_count": ([_VP, ctypes.POINTER(sph_particles), ctypes.c_double, _VP], ctypes.c_int),
            "sph_batch_create": ([ctypes.POINTER(_VP), ctypes.POINTER(sph_particles), ctypes.c_int32, _VP,
                                  ctypes.POINTER(_VP)], ctypes.c_int),
            "sph_batch_destroy": ([_VP], ctypes.c_int),
            "sph_batch_set_mode": ([_VP, ctypes.c_int32], ctypes.c_int),
            "sph_batch_set_count_block": ([_VP, ctypes.c_int32], ctypes.c_int),
            "sph_batch_set_gather": ([_VP, ctypes.c_int32], ctypes.c_int),
            "sph_batch_get_config": ([_VP, _I32, _I32, _I32], ctypes.c_int),
            "sph_batch_step": ([_VP], ctypes.c_int),
            "sph_batch_results": ([_VP, ctypes.POINTER(sph_result)], ctypes.c_int),
            "sph_batch_tune": ([_VP, ctypes.c_int32, ctypes.c_char_p, _I32, _I32, _D], ctypes.c_int),
            "sph_profile_read": ([_VP, _D, _I64, ctypes.c_int32], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _d3(v) -> ctypes.Array:
    a = list(v) + [0.0] * (3 - len(v))
    return (ctypes.c_double * 3)(*[float(x) for x in a[:3]])


def _d9(m) -> ctypes.Array:
    a = np.asarray(m, dtype=np.float64).reshape(9)
    return (ctypes.c_double * 9)(*[float(x) for x in a])


def check(status: int, what: str = "sphbuf") -> None:
    if status != SPH_OK:
        raise SphError(status, what)


# ------------------------------------------------------------------ C names ---

def sph_status_str(status: int) -> str:
    return lib().sph_status_str(int(status)).decode()


def sph_create(dim: int, lo, hi, cell_size: float, dp: float, capacity: int, max_events: int = 4096,
               next_id: int = 0, stream: int = 0, brick_log2: int = 0,
               brick_margin: int = 1, update_path: int = SPH_UPDATE_MERGED,
               build_method: int = SPH_BUILD_AUTO) -> Tuple[int, Optional[int]]:
    cfg = sph_config()
    cfg.dim = dim
    cfg.lo = _d3(lo)
    cfg.hi = _d3(hi)
    cfg.cell_size = cell_size
    cfg.dp = dp
    cfg.capacity = capacity
    cfg.max_events = max_events
    cfg.next_id = next_id
    cfg.stream = stream or None
    cfg.brick_log2 = brick_log2
    cfg.brick_margin = brick_margin
    cfg.update_path = int(update_path)
    cfg.build_method = int(build_method)
    out = _VP()
    st = lib().sph_create(ctypes.byref(cfg), ctypes.byref(out))
    if st == SPH_OK and out.value:
        _live_ctx.add(out.value)
    return st, out.value


def sph_destroy(ctx: int) -> int:
    """Destroys a context made by sph_create; a handle that is not alive (already
    destroyed, e.g. by the exit hook) is refused with SPH_ERR_ARG, never freed twice."""
    if ctx not in _live_ctx:
        return SPH_ERR_ARG
    _live_ctx.discard(ctx)
    return lib().sph_destroy(ctx)


def sph_buffer_define(ctx: int, kind: int, origin, rot, half, margin: float) -> Tuple[int, int]:
    bid = ctypes.c_int32(0)
    st = lib().sph_buffer_define(ctx, int(kind), _d3(origin), _d9(rot), _d3(half), float(margin), ctypes.byref(bid))
    return st, bid.value


def sph_grid_fit(ctx: int, p: sph_particles) -> int:
    return lib().sph_grid_fit(ctx, ctypes.byref(p))


def sph_celllist_build(ctx: int, p: sph_particles) -> int:
    return lib().sph_celllist_build(ctx, ctypes.byref(p))


def sph_set_fields(ctx: int, vel: Sequence[int], rho: int = -1) -> int:
    f = sph_fields()
    v = list(vel) + [-1] * (3 - len(vel))
    for i in range(3):
        f.vel[i] = int(v[i])
    f.rho = int(rho)
    return lib().sph_set_fields(ctx, ctypes.byref(f))


def sph_buffer_set_bc(ctx: int, buffer_id: int, kind: int, profile: int = SPH_PROFILE_PLUG, u: float = 0.0,
                      radius: float = 1.0, p_b: float = 0.0, rho0: float = 1.0, c0: float = 1.0) -> int:
    b = sph_bc()
    b.kind, b.profile = int(kind), int(profile)
    b.u, b.radius, b.p_b, b.rho0, b.c0 = float(u), float(radius), float(p_b), float(rho0), float(c0)
    return lib().sph_buffer_set_bc(ctx, int(buffer_id), ctypes.byref(b))


def sph_buffer_apply_bc(ctx: int, p: sph_particles) -> int:
    return lib().sph_buffer_apply_bc(ctx, ctypes.byref(p))


def sph_neighbor_count(ctx: int, p: sph_particles, radius: float, counts_ptr: int) -> int:
    """counts_ptr: device int32 array of at least N entries (async, on the context's stream)."""
    return lib().sph_neighbor_count(ctx, ctypes.byref(p), float(radius), _VP(counts_ptr))


def sph_buffer_rotate(ctx: int, p: sph_particles, buffer_id: int, center: Sequence[float], m) -> int:
    c = np.zeros(3)
    c[: len(center)] = center
    mm = np.ascontiguousarray(m, dtype=np.float64).reshape(9)
    return lib().sph_buffer_rotate(ctx, ctypes.byref(p), int(buffer_id), c.ctypes.data_as(_D), mm.ctypes.data_as(_D))


def sph_buffer_rotate_async(ctx: int, p: sph_particles, buffer_id: int, center: Sequence[float], m) -> int:
    c = np.zeros(3)
    c[: len(center)] = center
    mm = np.ascontiguousarray(m, dtype=np.float64).reshape(9)
    return lib().sph_buffer_rotate_async(ctx, ctypes.byref(p), int(buffer_id), c.ctypes.data_as(_D),
                                         mm.ctypes.data_as(_D))


def sph_buffer_apply_bc_async(ctx: int, p: sph_particles) -> int:
    return lib().sph_buffer_apply_bc_async(ctx, ctypes.byref(p))


def sph_last_bc_status(ctx: int) -> int:
    return lib().sph_last_bc_status(ctx)


def sph_buffer_cover(ctx: int, buffer_id: int, cap: int = 1 << 22):
    f = np.zeros(max(1, cap), dtype=np.int32)
    ln = np.zeros(max(1, cap), dtype=np.int32)
    n = ctypes.c_int64(0)
    st = lib().sph_buffer_cover(ctx, int(buffer_id), f.ctypes.data_as(_I32), ln.ctypes.data_as(_I32), int(cap),
                                ctypes.byref(n))
    return st, f[: n.value].copy(), ln[: n.value].copy()


def sph_celllist_build_noalloc(dim: int, lo, cell_size: float, dims, x_ptr: int, y_ptr: int, z_ptr: int,
                               n_dev_ptr: int, capacity: int, cell_start_ptr: int, cell_idx_ptr: int,
                               stream: int = 0) -> int:
    """Device pointers throughout (async on stream)."""
    d3 = (ctypes.c_int32 * 3)(*[int(v) for v in (list(dims) + [1, 1, 1])[:3]])
    return lib().sph_celllist_build_noalloc(int(dim), _d3(lo), float(cell_size), d3, _VP(x_ptr), _VP(y_ptr),
                                            _VP(z_ptr or None), _VP(n_dev_ptr), int(capacity), _VP(cell_start_ptr),
                                            _VP(cell_idx_ptr), _VP(stream or None))


def sph_buffer_identify(ctx: int, p: sph_particles, buffer_id: int = -1) -> int:
    return lib().sph_buffer_identify(ctx, ctypes.byref(p), int(buffer_id))


def sph_buffer_update(ctx: int, p: sph_particles) -> Tuple[int, int, int]:
    g, d = ctypes.c_int64(0), ctypes.c_int64(0)
    st = lib().sph_buffer_update(ctx, ctypes.byref(p), ctypes.byref(g), ctypes.byref(d))
    return st, g.value, d.value


def sph_buffer_update_async(ctx: int, p: sph_particles) -> int:
    return lib().sph_buffer_update_async(ctx, ctypes.byref(p))


def sph_buffer_update_fullscan(ctx: int, p: sph_particles) -> Tuple[int, int, int]:
    g, d = ctypes.c_int64(0), ctypes.c_int64(0)
    st = lib().sph_buffer_update_fullscan(ctx, ctypes.byref(p), ctypes.byref(g), ctypes.byref(d))
    return st, g.value, d.value


def sph_buffer_update_fullscan_async(ctx: int, p: sph_particles) -> int:
    return lib().sph_buffer_update_fullscan_async(ctx, ctypes.byref(p))


def sph_last_result(ctx: int) -> Tuple[int, sph_result]:
    r = sph_result()
    st = lib().sph_last_result(ctx, ctypes.byref(r))
    return st, r


def sph_last_events(ctx: int, cap: int) -> Tuple[int, np.ndarray, np.ndarray]:
    gen = np.zeros(max(1, cap), dtype=np.int64)
    dele = np.zeros(max(1, cap), dtype=np.int64)
    ng, nd = ctypes.c_int64(0), ctypes.c_int64(0)
    st = lib().sph_last_events(ctx, gen.ctypes.data_as(_I64), dele.ctypes.data_as(_I64), int(cap), ctypes.byref(ng),
                               ctypes.byref(nd))
    return st, gen[: min(cap, ng.value)].copy(), dele[: min(cap, nd.value)].copy()


def sph_build_stats(ctx: int):
    """(status, method of the last build, [us counting, us bucketed], [samples
    counting, samples bucketed]) -- the automatic method choice's view."""
    m = ctypes.c_int32()
    us = (ctypes.c_double * 2)()
    ns = (ctypes.c_int64 * 2)()
    st = lib().sph_build_stats(ctx, ctypes.byref(m), us, ns)
    return st, m.value, [us[0], us[1]], [ns[0], ns[1]]


def sph_build_retune(ctx: int) -> int:
    return lib().sph_build_retune(ctx)


def sph_celllist_view(ctx: int):
    cs, ci = _VP(), _VP()
    nc = ctypes.c_int64(0)
    dims = (ctypes.c_int32 * 3)()
    st = lib().sph_celllist_view(ctx, ctypes.byref(cs), ctypes.byref(ci), ctypes.byref(nc), dims)
    return st, cs.value, ci.value, nc.value, tuple(dims)


def sph_state_get(ctx: int) -> Tuple[int, int, np.ndarray]:
    nid = ctypes.c_int64(0)
    nl = np.zeros(SPH_MAX_BUFFERS, dtype=np.int64)
    st = lib().sph_state_get(ctx, ctypes.byref(nid), nl.ctypes.data_as(_I64))
    return st, nid.value, nl


def sph_state_set(ctx: int, next_id: int, n_labelled) -> int:
    nl = np.zeros(SPH_MAX_BUFFERS, dtype=np.int64)
    nl[: len(n_labelled)] = n_labelled
    return lib().sph_state_set(ctx, int(next_id), nl.ctypes.data_as(_I64))


def sph_state_export(ctx: int) -> Tuple[int, bytes]:
    buf = ctypes.create_string_buffer(SPH_STATE_BLOB_BYTES)
    n = ctypes.c_size_t(SPH_STATE_BLOB_BYTES)
    st = lib().sph_state_export(ctx, ctypes.cast(buf, _VP), ctypes.byref(n))
    return st, buf.raw[: n.value]


def sph_state_import(ctx: int, blob: bytes) -> int:
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    return lib().sph_state_import(ctx, ctypes.cast(buf, _VP), len(blob))


def sph_rotation_2d(theta: float) -> Tuple[int, np.ndarray]:
    r = (ctypes.c_double * 9)()
    st = lib().sph_rotation_2d(float(theta), r)
    return st, np.array(r[:]).reshape(3, 3)


def sph_rotation_axis_angle(n, theta: float) -> Tuple[int, np.ndarray]:
    r = (ctypes.c_double * 9)()
    st = lib().sph_rotation_axis_angle(_d3(n), float(theta), r)
    return st, np.array(r[:]).reshape(3, 3)


def sph_rotation_from_direction(d) -> Tuple[int, np.ndarray]:
    r = (ctypes.c_double * 9)()
    st = lib().sph_rotation_from_direction(_d3(d), r)
    return st, np.array(r[:]).reshape(3, 3)


def sph_check_rotation(dim: int, rot) -> int:
    return lib().sph_check_rotation(int(dim), _d9(rot))


def sph_grid_cover(dim: int, lo, cell_size: float, dims, origin, rot, half, margin: float, cap: int = 1 << 20):
    f = np.zeros(max(1, cap), dtype=np.int32)
    ln = np.zeros(max(1, cap), dtype=np.int32)
    n = ctypes.c_int64(0)
    d3 = (ctypes.c_int32 * 3)(*[int(x) for x in (list(dims) + [1, 1, 1])[:3]])
    st = lib().sph_grid_cover(int(dim), _d3(lo), float(cell_size), d3, _d3(origin), _d9(rot), _d3(half),
                              float(margin), f.ctypes.data_as(_I32), ln.ctypes.data_as(_I32), int(cap),
                              ctypes.byref(n))
    return st, f[: n.value].copy(), ln[: n.value].copy()


def sph_guard_band(dim: int, origin, half, margin: float, cell_size: float, dp: float) -> float:
    return lib().sph_guard_band(int(dim), _d3(origin), _d3(half), float(margin), float(cell_size), float(dp))


def sph_profile_enable(ctx: int, on: bool) -> int:
    return lib().sph_profile_enable(ctx, 1 if on else 0)


def sph_profile_read(ctx: int, reset: bool = False):
    ms = np.zeros(SPH_NPHASE)
    n = np.zeros(SPH_NPHASE, dtype=np.int64)
    st = lib().sph_profile_read(ctx, ms.ctypes.data_as(_D), n.ctypes.data_as(_I64), 1 if reset else 0)
    return st, ms, n


def sph_batch_create(ctxs, parts, stream: int = 0):
    n = len(ctxs)
    arr = (_VP * n)(*ctxs)
    parr = (sph_particles * n)(*parts)
    out = _VP()
    st = lib().sph_batch_create(arr, parr, n, stream or None, ctypes.byref(out))
    if st == SPH_OK and out.value:
        _live_batch.add(out.value)
    return st, out.value


def sph_batch_destroy(b: int) -> int:
    """As sph_destroy, for batches."""
    if b not in _live_batch:
        return SPH_ERR_ARG
    _live_batch.discard(b)
    return lib().sph_batch_destroy(b)


def sph_batch_profile_enable(b: int, on: bool) -> int:
    return lib().sph_batch_profile_enable(b, 1 if on else 0)


def sph_batch_profile_read(b: int, reset: bool = False):
    ms = np.zeros(5)
    n = np.zeros(5, dtype=np.int64)
    st = lib().sph_batch_profile_read(b, ms.ctypes.data_as(_D), n.ctypes.data_as(_I64), 1 if reset else 0)
    return st, ms, n


def sph_batch_graph_capture(b: int) -> int:
    return lib().sph_batch_graph_capture(b)


def sph_batch_graph_launch(b: int) -> int:
    return lib().sph_batch_graph_launch(b)


def sph_batch_set_mode(b: int, mode: int) -> int:
    return lib().sph_batch_set_mode(b, int(mode))


def sph_batch_set_count_block(b: int, ppb: int) -> int:
    return lib().sph_batch_set_count_block(b, int(ppb))


def sph_batch_set_gather(b: int, runs_per_block: int) -> int:
    return lib().sph_batch_set_gather(b, int(runs_per_block))


def sph_batch_get_config(b: int):
    """(status, mode, particles per count block, runs per classify workgroup)."""
    m, ppb, rpb = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    st = lib().sph_batch_get_config(b, ctypes.byref(m), ctypes.byref(ppb), ctypes.byref(rpb))
    return st, m.value, ppb.value, rpb.value


def sph_batch_step(b: int) -> int:
    return lib().sph_batch_step(b)


def sph_batch_results(b: int, n: int):
    res = (sph_result * n)()
    st = lib().sph_batch_results(b, res)
    return st, list(res)


def sph_batch_tune(b: int, trials: int = 5, cache_path: Optional[str] = None):
    mode, ppb, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0)
    st = lib().sph_batch_tune(b, int(trials), cache_path.encode() if cache_path else None, ctypes.byref(mode),
                              ctypes.byref(ppb), ctypes.byref(ms))
    return st, mode.value, ppb.value, ms.value


# ------------------------------------------------------------- marshalling ---

def particles_from_tensors(pos: Sequence, carried: Sequence, label, ids, n_dev) -> sph_particles:
    """Fill an sph_particles from torch device tensors (all of one capacity)."""
    p = sph_particles()
    cap = int(label.shape[0])
    for c, t in enumerate(pos):
        assert t.is_contiguous() and t.shape[0] == cap and str(t.dtype) == "torch.float32"
        p.pos[c] = t.data_ptr()
    assert len(carried) <= SPH_MAX_CARRIED
    for f, t in enumerate(carried):
        assert t.is_contiguous() and t.shape[0] == cap and str(t.dtype) == "torch.float32"
        p.carried[f] = t.data_ptr()
    p.n_carried = len(carried)
    assert str(label.dtype) == "torch.int32" and str(ids.dtype) == "torch.int64" and str(n_dev.dtype) == "torch.int64"
    p.label = label.data_ptr()
    p.id = ids.data_ptr()
    p.n_dev = n_dev.data_ptr()
    p.capacity = cap
    return p
