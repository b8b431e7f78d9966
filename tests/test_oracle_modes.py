"""The oracle's CPU-baseline modes against its brute-force update: the paper's
method on the CPU (candidates only from the cells of a cell list near each check
region) and the brute force on one thread and on all host threads.  Both must
give the brute force's events, arrays and labelled counts."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from tests._support import make_state, oracle_buffers, oracle_state


def _grid(wl):
    dims = [int(math.ceil((wl.hi[c] - wl.lo[c]) / wl.cell_size)) for c in range(wl.dim)]
    return np.float32(wl.lo[: wl.dim]), np.float32(1.0 / wl.cell_size), dims


def _local_step(wl, bufs, st, nl):
    lo32, inv, dims = _grid(wl)
    n = st.n
    start, idx = oracle.cell_list(wl.dim, lo32, inv, dims, st.pos[0][:n], st.pos[1][:n],
                                  st.pos[2][:n] if wl.dim == 3 else None)
    return oracle.update_local(bufs, st, lo32, inv, dims, start, idx, nl)


def _same(a: oracle.State, b: oracle.State, what):
    assert a.n == b.n and a.next_id == b.next_id, what
    n = a.n
    for x, y in zip(a.pos + a.carried + [a.label, a.id], b.pos + b.carried + [b.label, b.id]):
        np.testing.assert_array_equal(x[:n], y[:n], err_msg=what)


@pytest.mark.parametrize("name,steps", [("channel2d", 200), ("bent_channel2d", 40), ("pipe3d", 30),
                                        ("tree3d", 60)])
def test_local_cell_mode_equals_brute_force(name, steps):
    wl = {"channel2d": W.channel2d, "bent_channel2d": W.bent_channel2d,
          "pipe3d": lambda: W.pipe3d(dp=0.004), "tree3d": lambda: W.tree3d(dp=0.004)}[name]()
    bufs = oracle_buffers(wl)
    ref = oracle_state(wl)
    loc = oracle_state(wl)
    assert oracle.identify(bufs, ref, -1)[0] == 0
    rc, nl = oracle.identify(bufs, loc, -1)
    assert rc == 0
    total = 0
    for step in range(steps):
        W.advect_host(wl, ref.pos, ref.n, step)
        W.advect_host(wl, loc.pos, loc.n, step)
        r = oracle.update(bufs, ref)
        q = _local_step(wl, bufs, loc, nl)
        assert r.status == q.status == 0, (step, r.status, q.status)
        np.testing.assert_array_equal(q.gen, r.gen)
        np.testing.assert_array_equal(q.dele, r.dele)
        np.testing.assert_array_equal(q.n_labelled, r.n_labelled)
        _same(ref, loc, f"{name} step {step}")
        nl = q.n_labelled
        total += len(r.gen) + len(r.dele)
    assert total > 0


def test_local_cell_mode_reports_a_buffer_particle_outside_its_region():
    I3 = np.eye(3)
    bufs = [oracle.Buffer(oracle.INLET, (0.5, 0.5, 0), I3, (0.5, 0.5, 0), 0.25),
            oracle.Buffer(oracle.OUTLET, (4.5, 0.5, 0), I3, (0.5, 0.5, 0), 0.25)]
    st = make_state(2, [(0.5, 0.5), (2.5, 0.5), (4.4, 0.4)], labels=[1, 1, 2])
    lo32, inv, dims = np.float32([-1, -1]), np.float32(1 / 0.3), [25, 10]
    start, idx = oracle.cell_list(2, lo32, inv, dims, st.pos[0][:3], st.pos[1][:3])
    before = st.copy()
    q = oracle.update_local(bufs, st, lo32, inv, dims, start, idx, [2, 1])
    assert q.status == oracle.ERR_CFL
    assert oracle.update(bufs, before.copy()).status == oracle.ERR_CFL
    for x, y in zip(st.pos + [st.label, st.id], before.pos + [before.label, before.id]):
        np.testing.assert_array_equal(x, y)


def test_brute_force_is_the_same_on_one_and_all_threads():
    wl = W.pipe3d(dp=0.004)
    bufs = oracle_buffers(wl)
    a, b = oracle_state(wl), oracle_state(wl)
    oracle.identify(bufs, a, -1)
    oracle.identify(bufs, b, -1)
    n_all = oracle.set_threads(0)
    try:
        for step in range(20):
            W.advect_host(wl, a.pos, a.n, step)
            W.advect_host(wl, b.pos, b.n, step)
            assert oracle.set_threads(1) == 1
            ra = oracle.update(bufs, a)
            oracle.set_threads(n_all)
            rb = oracle.update(bufs, b)
            assert ra.status == rb.status == 0
            np.testing.assert_array_equal(ra.gen, rb.gen)
            np.testing.assert_array_equal(ra.dele, rb.dele)
            _same(a, b, f"step {step}")
        # the first error by index is reported, whatever the threads
        c = a.copy()
        lab = np.flatnonzero(c.label[: c.n] > 0)
        c.pos[0][lab[-1]] = np.float32(1e3)      # a buffer particle far out of its region (CFL) ...
        c.pos[1][lab[0]] = np.float32(np.nan)    # ... and a non-finite position
        assert oracle.update(bufs, c.copy()).status == oracle.ERR_NONFINITE
        c.pos[1][lab[0]] = np.float32(0.0)
        oracle.set_threads(1)
        s1 = oracle.update(bufs, c.copy()).status
        oracle.set_threads(n_all)
        assert s1 == oracle.update(bufs, c.copy()).status == oracle.ERR_CFL
    finally:
        oracle.set_threads(n_all)
