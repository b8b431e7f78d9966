"""GPU-side helpers for the parity tests: a library Domain fed with the same seeded
inputs (and the oracle's own frames) as the FP64 oracle, plus comparisons."""
from __future__ import annotations

from typing import Sequence

import numpy as np

import oracle
from tests._support import oracle_state

# Update path of the contexts the tests make ("merged", the library's default, or
# "cells") and their cell-list build method ("auto", the default, "counting" or
# "bucketed"); tests of one path or method set them with monkeypatch.setattr.
UPDATE_PATH = "merged"
BUILD_METHOD = "auto"


def make_domain_raw(dim, lo, hi, cell_size, dp, bufs: Sequence[oracle.Buffer], st: oracle.State,
                    max_events: int = 4096, brick_log2: int = 0, brick_margin: int = 1, update_path: str = None,
                    build_method: str = None):
    from paper_2406_16786_amd.domain import Domain
    d = Domain(dim, lo, hi, cell_size, dp, st.capacity, st.pos, st.carried, st.label, st.id, st.n, st.next_id,
               max_events=max_events, brick_log2=brick_log2, brick_margin=brick_margin,
               update_path=update_path or UPDATE_PATH, build_method=build_method or BUILD_METHOD)
    for b in bufs:
        d.define(b.kind, b.origin, b.rot, b.half, b.margin)
    if brick_log2:
        d.fit()
    return d


def make_domain(wl, bufs: Sequence[oracle.Buffer], st: oracle.State = None, max_events: int = 4096,
                cell_size: float = None, lo=None, hi=None, brick_log2: int = 0, brick_margin: int = 1):
    st = st if st is not None else oracle_state(wl)
    return make_domain_raw(wl.dim, lo if lo is not None else wl.lo, hi if hi is not None else wl.hi,
                           cell_size if cell_size is not None else wl.cell_size, wl.dp, bufs, st, max_events,
                           brick_log2, brick_margin)


def upload_state(d, st: oracle.State) -> None:
    d.upload(st.pos, st.carried, st.label, st.id, st.n)


def assert_same_state(d, st: oracle.State, what: str = "") -> None:
    pos, car, lab, ids, n = d.download()
    assert n == st.n, f"{what}: n {n} != {st.n}"
    for c in range(st.dim):
        np.testing.assert_array_equal(pos[c][:n], st.pos[c][:n], err_msg=f"{what}: pos[{c}]")
    for f in range(len(st.carried)):
        np.testing.assert_array_equal(car[f][:n], st.carried[f][:n], err_msg=f"{what}: carried[{f}]")
    np.testing.assert_array_equal(lab[:n], st.label[:n], err_msg=f"{what}: label")
    np.testing.assert_array_equal(ids[:n], st.id[:n], err_msg=f"{what}: id")


def advect_device(wl, d, step: int, gen) -> None:
    """x <- x + u dt on the GPU with the workload's prescribed velocity (seeded
    noise from a torch generator): the harness's move between two updates of a
    long full-size run.  The oracle is then fed the GPU's own pre-update states."""
    import torch
    n = d.n()
    gen.manual_seed(wl.seed_noise + step)
    with torch.cuda.stream(d.stream):
        p = [t[:n] for t in d.pos]
        noise = torch.randn((wl.dim, n), generator=gen, device=d.device, dtype=torch.float32)
        u = wl.velocity(torch, p, step, noise)
        for c in range(wl.dim):
            p[c].add_(u[c] * wl.dt)
    d.stream.synchronize()


def host_state(d, n_carried_kept=None) -> oracle.State:
    """Host copy of a domain's live state (all carried fields, or the first
    n_carried_kept of them) as an oracle State with the library's next_id."""
    from paper_2406_16786_amd import sphbuf as S
    d.stream.synchronize()
    n = int(d.n_dev.item())
    pos = [t.cpu().numpy() for t in d.pos]
    car = [t.cpu().numpy() for t in d.carried[: n_carried_kept]] if n_carried_kept != 0 else []
    lab = d.label.cpu().numpy()
    ids = d.id.cpu().numpy()
    nid = int(S.sph_state_get(d.ctx)[1])
    return oracle.State(len(pos), pos, car, lab, ids, n, nid)
