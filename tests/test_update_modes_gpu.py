"""The two update paths behind the same C ABI against the FP64 oracle: the update
that walks the cover cells of the finished cell list (the default) and the
overlapped step (SPHBUF_UPDATE=overlap: the count pass gathers the particles of the
buffers' cover cells, the update runs on them while the scan and scatter finish on a
side stream); plus the call orders the overlapped step has to survive."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests._gpu import assert_same_state, make_domain, upload_state
from tests._support import oracle_buffers, oracle_state
from tests.test_parity_gpu import _cell_list, _run_steps

pytestmark = pytest.mark.gpu


def _mode(monkeypatch, mode):
    if mode == "overlap":
        monkeypatch.setenv("SPHBUF_UPDATE", "overlap")
    else:
        monkeypatch.delenv("SPHBUF_UPDATE", raising=False)


@pytest.mark.parametrize("mode", ["overlap", "cells"])
def test_channel_and_pipe(mode, monkeypatch):
    _mode(monkeypatch, mode)
    g, dl = _run_steps(W.channel2d(), 120)
    assert g > 0 and dl > 0
    g, dl = _run_steps(W.pipe3d(dp=0.004), 25, check_every=5)
    assert g > 0


@pytest.mark.parametrize("mode", ["overlap", "cells"])
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


def test_unconsumed_builds_and_interleaved_calls(monkeypatch):
    """Overlapped step: a build no update consumed (its candidates must not count
    twice), a full-scan update after such a build, a neighbour search and a
    cell-list view between the build and the update."""
    _mode(monkeypatch, "overlap")
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


def test_overlapped_step_full_size(monkeypatch):
    """The overlapped step on the benchmark's pipe (7.86 M particles), two steps."""
    _mode(monkeypatch, "overlap")
    _run_steps(W.pipe3d(), 2)
