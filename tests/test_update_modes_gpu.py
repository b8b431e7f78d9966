"""The two update paths behind the same C ABI against the FP64 oracle: the merged
step (SPH_UPDATE_MERGED, the default: the count pass classifies the particles of
the buffers' cover cells and emits their events, the update runs the finalize
beside the scan tiles, then the scatter) and the update that walks the cover
cells of the finished cell list (SPH_UPDATE_CELLS); plus the call orders the
merged step has to survive."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests._gpu import assert_same_state, make_domain, upload_state
from tests._support import oracle_buffers, oracle_state
from tests.test_parity_gpu import _cell_list, _run_steps

pytestmark = pytest.mark.gpu


def _mode(monkeypatch, mode):
    import tests._gpu as G
    monkeypatch.setattr(G, "UPDATE_PATH", mode)


@pytest.mark.parametrize("mode", ["merged", "cells"])
def test_channel_and_pipe(mode, monkeypatch):
    _mode(monkeypatch, mode)
    g, dl = _run_steps(W.channel2d(), 120)
    assert g > 0 and dl > 0
    g, dl = _run_steps(W.pipe3d(dp=0.004), 25, check_every=5)
    assert g > 0


@pytest.mark.parametrize("mode", ["merged", "cells"])
def test_tree_bidirectional_sparse_grid(mode, monkeypatch):
    _mode(monkeypatch, mode)
    g, dl = _run_steps(W.tree3d(dp=0.004), 60, check_every=20, brick_log2=3)
    assert g > 0 and dl > 0


def _setup(wl):
    bufs = oracle_buffers(wl)
    st = oracle_state(wl)
    d = make_domain(wl, bufs, st)
    assert oracle.identify(bufs, st, -1)[0] == 0 and d.identify(-1) == 0
    return bufs, st, d


def _check_update(d, bufs, st, what):
    gst, g, dl = d.update()
    res = oracle.update(bufs, st)
    assert gst == res.status == 0, (what, gst, res.status)
    _, gg, dd = d.events()
    np.testing.assert_array_equal(gg, res.gen, err_msg=what)
    np.testing.assert_array_equal(dd, res.dele, err_msg=what)
    assert_same_state(d, st, what)


@pytest.mark.parametrize("mode", ["merged", "cells"])
def test_unconsumed_builds_and_interleaved_calls(mode, monkeypatch):
    """A build no update consumed (its events must not count twice),
    a full-scan update after such a build, a neighbour search and a cell-list view
    between the build and the update."""
    _mode(monkeypatch, mode)
    wl = W.channel2d()
    bufs, st, d = _setup(wl)
    for step in range(40):
        W.advect_host(wl, st.pos, st.n, step)
        upload_state(d, st)
        kind = step % 4
        if kind == 0:
            d.build()
            d.build()
            _check_update(d, bufs, st, f"step {step}: two builds")
        elif kind == 1:
            d.build()
            gst, g, dl = d.update_fullscan()
            res = oracle.update(bufs, st)
            assert gst == res.status == 0
            assert_same_state(d, st, f"step {step}: full scan after an unconsumed build")
        elif kind == 2:
            d.build()
            st_nb, counts = d.neighbor_count(wl.cell_size)
            assert st_nb == 0
            n = st.n
            np.testing.assert_array_equal(counts.cpu().numpy()[:n],
                                          oracle.neighbor_count(2, st.pos[0][:n], st.pos[1][:n], None, wl.cell_size))
            _check_update(d, bufs, st, f"step {step}: neighbour search before the update")
        else:
            d.build()
            cs, ci, dims = _cell_list(d, st.n)
            n = st.n
            ref_s, ref_i = oracle.cell_list(2, np.float32(wl.lo[:2]), np.float32(1.0 / wl.cell_size), dims[:2],
                                            st.pos[0][:n], st.pos[1][:n])
            np.testing.assert_array_equal(cs, ref_s)
            _check_update(d, bufs, st, f"step {step}: cell-list view before the update")
    d.close()


def test_cover_walk_full_size(monkeypatch):
    """The cover-cell walk on the benchmark's pipe (7.86 M particles), two steps
    (the parity tests run the merged step, the default)."""
    _mode(monkeypatch, "cells")
    _run_steps(W.pipe3d(), 2)


def test_merged_step_cell_list_after_the_update(monkeypatch):
    """The scatter of a merged step runs after the finalize has changed the live
    count: the cell list it leaves is that of the state the build saw."""
    _mode(monkeypatch, "merged")
    wl = W.channel2d()
    bufs, st, d = _setup(wl)
    dims = _cell_list(d, 0)[2]
    for step in range(30):
        W.advect_host(wl, st.pos, st.n, step)
        upload_state(d, st)
        n = st.n
        ref_s, ref_i = oracle.cell_list(2, np.float32(wl.lo[:2]), np.float32(1.0 / wl.cell_size), dims[:2],
                                        st.pos[0][:n].copy(), st.pos[1][:n].copy())
        d.build()
        _check_update(d, bufs, st, f"step {step}")
        cs, ci, _ = _cell_list(d, n)
        np.testing.assert_array_equal(cs, ref_s, err_msg=f"step {step}")
        for c in np.flatnonzero(np.diff(ref_s)):  # each cell's set (the order inside a cell is free)
            np.testing.assert_array_equal(np.sort(ci[ref_s[c]:ref_s[c + 1]]), np.sort(ref_i[ref_s[c]:ref_s[c + 1]]))
    d.close()


@pytest.mark.parametrize("case", ["vipo_pipe3d", "pivo_channel2d"])
def test_cover_walk_with_boundary_conditions(case, monkeypatch):
    """The boundary-condition runs on the cover-cell walk.  (On the merged path, the
    default, boundary conditions applied between the build and the update drop the
    build's events and the update walks the cover cells.)"""
    from tests.test_bc_gpu import test_boundary_conditions_over_steps
    _mode(monkeypatch, "cells")
    test_boundary_conditions_over_steps(case)


def test_cover_walk_sprinkler(monkeypatch):
    from tests.test_bc_gpu import test_sprinkler_rotating_inlet
    _mode(monkeypatch, "cells")
    test_sprinkler_rotating_inlet()


@pytest.mark.parametrize("what", ["cfl", "capacity", "nonfinite", "empty", "all_deleted", "hand", "unaligned",
                                  "clustered", "guard"])
def test_cover_walk_edge_cases(what, monkeypatch):
    import tests.test_parity_gpu as P
    _mode(monkeypatch, "cells")
    if what == "cfl":
        P.test_cfl_violation_leaves_state_untouched("local")
    elif what == "capacity":
        P.test_capacity_exhaustion_leaves_state_untouched("local")
    elif what == "nonfinite":
        P.test_nonfinite_position_leaves_state_untouched("local")
    elif what == "empty":
        P.test_empty_domain()
    elif what == "all_deleted":
        P.test_every_particle_deleted()
    elif what == "hand":
        for case in range(3):
            P.test_hand_examples_on_gpu(case, "local")
    elif what == "unaligned":
        P.test_unaligned_arrays_take_the_scalar_paths("local")
    elif what == "clustered":
        P.test_clustered_event_indices(200_000, "local")
    else:
        for dim in (2, 3):
            P.test_guard_band_decisions_equal_fp64(dim, 0)


def test_cover_walk_tree_full_size(monkeypatch):
    """The cover-cell walk on the branching network at full size (16.1 M particles,
    brick-sparse grid, four bidirectional buffers), two steps."""
    _mode(monkeypatch, "cells")
    _run_steps(W.tree3d(), 2, brick_log2=3)


def test_cover_walk_bent_channel_1000_steps(monkeypatch):
    """The cover-cell walk on the bent 2-D channel for its full 1,000 steps (events
    every step, every array every 100 steps)."""
    _mode(monkeypatch, "cells")
    g, dl = _run_steps(W.bent_channel2d(), 1000, check_every=100)
    assert g > 0 and dl > 0


@pytest.mark.parametrize("then", ["build", "fullscan"])
def test_merged_dropped_events_leave_no_nonfinite_flag(then, monkeypatch):
    """A merged build that met a non-finite position and whose events a library call
    dropped before any update: once the position is finite again, the next build's
    update (or a full-scan update) must not report it."""
    import tests.test_parity_gpu as P
    _mode(monkeypatch, "merged")
    wl, bufs, st = P._two_buffer_case([(1.125, 0.5), (np.nan, 0.4), (0.3, 0.3)], [1, 0, 1])
    d = make_domain(wl, bufs, st)
    P._identify_counts(d, bufs, st)
    d.build()                        # classifies, raises the non-finite flag
    d.set_fields([0, 1], -1)         # drops the build's events
    st.pos[0][1] = np.float32(0.4)   # finite again
    upload_state(d, st)
    if then == "build":
        d.build()
        gst, g, dl = d.update()
    else:
        gst, g, dl = d.update_fullscan()
    res = oracle.update(bufs, st)
    assert gst == res.status == 0, (gst, res.status)
    assert_same_state(d, st, "after the dropped build")
    d.close()
