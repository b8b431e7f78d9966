"""Glue between the seeded workloads and the FP64 oracle, shared by the tests."""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

import oracle
import workloads as W


def oracle_rotation(spec: W.BufferSpec, dim: int) -> np.ndarray:
    """Global->local matrix for a buffer placement, from the oracle's own frames."""
    if dim == 2:
        theta = spec.angle if spec.angle is not None else math.atan2(spec.direction[1], spec.direction[0])
        return oracle.rotation_2d(theta)
    return oracle.rotation_from_direction(spec.direction)


def oracle_buffers(wl_or_specs, dim: int = None) -> List[oracle.Buffer]:
    specs = wl_or_specs.buffers if hasattr(wl_or_specs, "buffers") else wl_or_specs
    d = dim if dim is not None else wl_or_specs.dim
    return [oracle.Buffer(s.kind, tuple(s.origin), oracle_rotation(s, d), tuple(s.half), s.margin)
            for s in specs]


def oracle_state(wl: W.Workload) -> oracle.State:
    return oracle.State(wl.dim, [p.copy() for p in wl.pos], [c.copy() for c in wl.carried],
                        wl.label.copy(), wl.id.copy(), wl.n, int(wl.n))


def make_state(dim: int, pts: np.ndarray, capacity: int = None, carried: int = 2,
               labels: Sequence[int] = None, next_id: int = None) -> oracle.State:
    """Host state from an (n, dim) array of positions; carried fields are 10*i + f."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, dim)
    n = pts.shape[0]
    cap = capacity if capacity is not None else n + 16
    pos = []
    for c in range(dim):
        a = np.zeros(cap, np.float32)
        a[:n] = pts[:, c].astype(np.float32)
        pos.append(a)
    car = []
    for f in range(carried):
        a = np.zeros(cap, np.float32)
        a[:n] = (10.0 * np.arange(n) + f).astype(np.float32)
        car.append(a)
    lab = np.zeros(cap, np.int32)
    if labels is not None:
        lab[:n] = labels
    ids = np.full(cap, -1, np.int64)
    ids[:n] = np.arange(n)
    return oracle.State(dim, pos, car, lab, ids, n, n if next_id is None else next_id)


def local(dim: int, buf: oracle.Buffer, st: oracle.State) -> np.ndarray:
    n = st.n
    return oracle.local_coords(dim, buf, st.pos[0][:n], st.pos[1][:n], st.pos[2][:n] if dim == 3 else None)


_KINDS = {"inlet": oracle.INLET, "outlet": oracle.OUTLET, "bidir": oracle.BIDIR}


def golden_cases(name: str = "hand_examples.json"):
    """Cases of a golden fixture under tests/golden/: (case dict, oracle buffers,
    fresh host state).  Frames come from the oracle's own constructions of the
    printed angle or direction."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    data = json.load(open(path))
    out = []
    for c in data["cases"]:
        bufs = []
        for b in c["buffers"]:
            rot = oracle.rotation_2d(b["angle"]) if "angle" in b else oracle.rotation_from_direction(b["direction"])
            bufs.append(oracle.Buffer(_KINDS[b["kind"]], tuple(b["origin"]), rot, tuple(b["half"]), b["margin"]))
        pts = [p["pos"] for p in c["particles"]]
        labels = [p["label"] for p in c["particles"]]
        st = make_state(c["dim"], pts, capacity=c["capacity"], labels=labels, next_id=c["next_id"], carried=3)
        out.append((c, bufs, st))
    return out
