"""GPU parity: the HIP library through its C ABI against the FP64 oracle.

Index sets of generated and deleted particles, labels, ids, counts and the whole
post-update particle arrays must be bit-identical to the oracle's (the library
takes every crossing decision inside the guard band in FP64 exactly as the
oracle does and recycles with the same FP64 expression, so recycled positions
match exactly, well inside the 1e-6 dp tolerance).
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
import workloads as W
from tests._gpu import assert_same_state, make_domain, make_domain_raw, upload_state
from tests._support import golden_cases, local, make_state, oracle_buffers, oracle_state

pytestmark = pytest.mark.gpu

I3 = np.eye(3)


def _hip():
    return ctypes.CDLL("libamdhip64.so")


def _d2h(dst: np.ndarray, src_ptr: int) -> None:
    hip = _hip()
    hip.hipDeviceSynchronize()
    rc = hip.hipMemcpy(ctypes.c_void_p(dst.ctypes.data), ctypes.c_void_p(src_ptr), ctypes.c_size_t(dst.nbytes), 2)
    assert rc == 0


def _cell_list(d, n):
    from paper_2406_16786_amd import sphbuf as S
    st, cs_ptr, ci_ptr, ncell, dims = S.sph_celllist_view(d.ctx)
    assert st == 0
    cs = np.zeros(ncell + 1, np.int32)
    ci = np.zeros(max(1, n), np.int32)
    _d2h(cs, cs_ptr)
    if n:
        _d2h(ci, ci_ptr)
    return cs, ci[:n], dims


def _run_steps(wl, steps, mode="local", identify=True, check_every=1, cell_size=None, brick_log2=0):
    bufs = oracle_buffers(wl)
    st = oracle_state(wl)
    d = make_domain(wl, bufs, st, cell_size=cell_size, brick_log2=brick_log2)
    if identify:
        rc_o, nl_o = oracle.identify(bufs, st, -1)
        assert d.identify(-1) == 0
        assert rc_o == 0
        assert_same_state(d, st, "identify")
    total_g = total_d = 0
    for step in range(steps):
        W.advect_host(wl, st.pos, st.n, step)
        upload_state(d, st)
        if mode == "local":
            d.build()
            gst, g, dl = d.update()
        else:
            gst, g, dl = d.update_fullscan()
        res = oracle.update(bufs, st)
        assert gst == res.status == 0, f"step {step}: gpu {gst} oracle {res.status}"
        eg, gg, dd = d.events()
        assert eg == 0
        np.testing.assert_array_equal(gg, res.gen, err_msg=f"step {step} generated")
        np.testing.assert_array_equal(dd, res.dele, err_msg=f"step {step} deleted")
        assert g == len(res.gen) and dl == len(res.dele)
        rs, r = d.result()
        assert rs == 0 and r.n_after == st.n and r.next_id == st.next_id
        assert list(r.n_labelled[: len(bufs)]) == list(res.n_labelled)
        if step % check_every == 0 or step == steps - 1:
            assert_same_state(d, st, f"step {step}")
        total_g += g
        total_d += dl
    d.close()
    return total_g, total_d


# ------------------------------------------------------------- cell list ---

@pytest.mark.parametrize("method", ["counting", "bucketed"])
@pytest.mark.parametrize("path", ["merged", "cells"])
@pytest.mark.parametrize("name", ["channel2d", "bent_channel2d", "pipe3d_small"])
def test_celllist_matches_oracle(name, path, method, monkeypatch):
    import tests._gpu as G
    monkeypatch.setattr(G, "UPDATE_PATH", path)
    monkeypatch.setattr(G, "BUILD_METHOD", method)
    wl = {"channel2d": W.channel2d, "bent_channel2d": W.bent_channel2d,
          "pipe3d_small": lambda: W.pipe3d(dp=0.004)}[name]()
    bufs = oracle_buffers(wl)
    d = make_domain(wl, bufs)
    d.build()
    cs, ci, dims = _cell_list(d, wl.n)
    lo32 = np.float32(wl.lo[: wl.dim])
    inv = np.float32(1.0 / wl.cell_size)
    ocs, oci = oracle.cell_list(wl.dim, lo32, inv, dims[: wl.dim], wl.pos[0][: wl.n], wl.pos[1][: wl.n],
                                wl.pos[2][: wl.n] if wl.dim == 3 else None)
    np.testing.assert_array_equal(cs, ocs)
    # order inside a cell depends on atomics: compare each cell's set
    assert np.array_equal(np.sort(ci), np.arange(wl.n))
    cell_of = np.repeat(np.arange(len(ocs) - 1), np.diff(ocs))
    got = ci[np.lexsort((ci, cell_of))]
    exp = oci[np.lexsort((oci, cell_of))]
    np.testing.assert_array_equal(got, exp)
    d.close()


@pytest.mark.parametrize("method", ["counting", "bucketed"])
def test_celllist_random_9_5m(method):
    """9.5 M random particles in a box (no buffer: the plain count pass)."""
    n = 9_500_000
    pos, car, lab, ids = W.random_box_particles(7, n, 3, (0, 0, 0), (1.0, 0.5, 0.5), capacity=n + 16, n_carried=1)
    st = oracle.State(3, pos, car, lab, ids, n, n)
    d = make_domain_raw(3, (0, 0, 0), (1.0, 0.5, 0.5), 0.01, 0.004, [], st, build_method=method)
    d.build()
    cs, ci, dims = _cell_list(d, n)
    ocs, oci = oracle.cell_list(3, np.float32([0, 0, 0]), np.float32(1.0 / 0.01), dims, pos[0][:n], pos[1][:n],
                                pos[2][:n])
    np.testing.assert_array_equal(cs, ocs)
    cell_of = np.repeat(np.arange(len(ocs) - 1), np.diff(ocs))
    np.testing.assert_array_equal(ci[np.lexsort((ci, cell_of))], oci)
    d.close()


def test_bucketed_builds_of_changing_particle_sets():
    """Bucketed builds of very different particle sets on one context (uniform,
    crowded into one corner, uniform again): nothing of one build's bucket layout
    or counts may leak into the next; every cell list equals the oracle's."""
    import torch
    n = 400_000
    rng = np.random.default_rng(31)
    pts_a = rng.uniform((0.0, 0.0, 0.0), (1.0, 0.5, 0.5), (n, 3))
    pts_b = rng.uniform((0.0, 0.0, 0.0), (0.3, 0.2, 0.1), (n, 3))
    st = make_state(3, pts_a, capacity=n + 16)
    d = make_domain_raw(3, (0, 0, 0), (1.0, 0.5, 0.5), 0.01, 0.004, [], st, build_method="bucketed")
    for pts in (pts_a, pts_b, pts_a):
        stp = make_state(3, pts, capacity=n + 16)
        with torch.cuda.stream(d.stream):
            for c in range(3):
                d.pos[c].copy_(torch.from_numpy(stp.pos[c][: n + 16]))
        d.stream.synchronize()
        d.build()
        cs, ci, dims = _cell_list(d, n)
        ocs, oci = oracle.cell_list(3, np.float32([0, 0, 0]), np.float32(1.0 / 0.01), dims, stp.pos[0][:n],
                                    stp.pos[1][:n], stp.pos[2][:n])
        np.testing.assert_array_equal(cs, ocs)
        cell_of = np.repeat(np.arange(len(ocs) - 1), np.diff(ocs))
        np.testing.assert_array_equal(ci[np.lexsort((ci, cell_of))], oci[np.lexsort((oci, cell_of))])
    d.close()


def test_celllist_buckets_of_4096_cells():
    """A 2-D grid of 16.4 M cells takes buckets of 4096 cells (the largest): each
    bucket's counting sort walks its cells in several rounds of its workgroup.
    3 M random particles against the oracle's cell list."""
    n = 3_000_000
    rng = np.random.default_rng(23)
    pts = rng.uniform((0.0, 0.0), (1.0, 4000.0 / 4096.0), (n, 2))
    st = make_state(2, pts, capacity=n + 16)
    cs_ = 1.0 / 4096.0
    d = make_domain_raw(2, (0, 0, 0), (1.0, 4000.0 / 4096.0, 0.0), cs_, cs_, [], st)
    d.build()
    cs, ci, dims = _cell_list(d, n)
    assert dims[0] * dims[1] > 4096 * 2048
    ocs, oci = oracle.cell_list(2, np.float32([0, 0]), np.float32(1.0 / cs_), dims[:2], st.pos[0][:n], st.pos[1][:n])
    np.testing.assert_array_equal(cs, ocs)
    cell_of = np.repeat(np.arange(len(ocs) - 1), np.diff(ocs))
    np.testing.assert_array_equal(ci[np.lexsort((ci, cell_of))], oci)
    d.close()


def test_celllist_full_size_network_repeatable():
    """The branching network at full size (16.1 M particles, brick-sparse grid,
    buckets of 1024 cells): repeated builds by each method through cover-walk
    contexts and one through a merged context give the same cell starts and the
    same particles in every cell (the order inside a cell is free)."""
    import tests._gpu as G
    wl = W.tree3d()
    bufs = oracle_buffers(wl)
    st = oracle_state(wl)
    n = st.n
    lists = []
    for path, method, builds in (("cells", "counting", 2), ("cells", "bucketed", 2), ("merged", "auto", 1)):
        old, oldm = G.UPDATE_PATH, G.BUILD_METHOD
        G.UPDATE_PATH, G.BUILD_METHOD = path, method
        try:
            d = make_domain(wl, bufs, st, brick_log2=3)
        finally:
            G.UPDATE_PATH, G.BUILD_METHOD = old, oldm
        for _ in range(builds):
            d.build()
            cs, ci, _ = _cell_list(d, n)
            cell_of = np.repeat(np.arange(len(cs) - 1), np.diff(cs))
            lists.append((cs, ci[np.lexsort((ci, cell_of))]))
        d.close()
    for cs, ci in lists[1:]:
        np.testing.assert_array_equal(cs, lists[0][0])
        np.testing.assert_array_equal(ci, lists[0][1])
    assert lists[0][0][-1] == n


def test_celllist_crowded_cell_on_a_fine_grid():
    """33 M cells leave 6 bits for the rank in the packed (key, rank) word, so
    500 particles in one cell take the full-width spill path of the build."""
    n_rand, n_crowd = 100_000, 500
    rng = np.random.default_rng(11)
    cs_ = 1.0 / 5800.0
    pts = np.concatenate([rng.uniform(0.0, 1.0, (n_rand, 2)),
                          (0.5 + 0.5 * cs_) + rng.uniform(-0.2 * cs_, 0.2 * cs_, (n_crowd, 2))])
    n = len(pts)
    st = make_state(2, pts, capacity=n + 16)
    d = make_domain_raw(2, (0, 0, 0), (1.0, 1.0, 0.0), cs_, cs_, [], st)
    d.build()
    cs, ci, dims = _cell_list(d, n)
    assert dims[0] * dims[1] > (1 << 25)
    ocs, oci = oracle.cell_list(2, np.float32([0, 0]), np.float32(1.0 / cs_), dims[:2], st.pos[0][:n], st.pos[1][:n],
                                None)
    np.testing.assert_array_equal(cs, ocs)
    assert np.diff(ocs).max() >= n_crowd
    cell_of = np.repeat(np.arange(len(ocs) - 1), np.diff(ocs))
    np.testing.assert_array_equal(ci[np.lexsort((ci, cell_of))], oci[np.lexsort((oci, cell_of))])
    d.close()


@pytest.mark.parametrize("method", ["counting", "bucketed"])
def test_celllist_cells_around_the_held_entries(method):
    """A grid of 3600 cells makes every cell a bucket of its own, so cells of 4095,
    4096 and 4097 particles sit on either side of the bucket sort's 4096 held
    entries (placed in LDS and stored in order up to there, stored one by one
    past it) and one of 9000 streams most of its entries; 50 k particles spread
    over the other cells.  Both builds against the oracle's cell list."""
    rng = np.random.default_rng(41)
    cs_ = 1.0 / 60.0
    crowds = {(7, 9): 4095, (30, 30): 4096, (31, 30): 4097, (52, 3): 9000}
    parts = [rng.uniform(0.0, 1.0, (50_000, 2))]
    for (ix, iy), m in crowds.items():
        ctr = np.array([(ix + 0.5) * cs_, (iy + 0.5) * cs_])
        parts.append(ctr + rng.uniform(-0.3 * cs_, 0.3 * cs_, (m, 2)))
    pts = np.concatenate(parts)
    pts = pts[rng.permutation(len(pts))]
    n = len(pts)
    st = make_state(2, pts, capacity=n + 16)
    d = make_domain_raw(2, (0, 0, 0), (1.0, 1.0, 0.0), cs_, cs_, [], st, build_method=method)
    d.build()
    cs, ci, dims = _cell_list(d, n)
    assert dims[0] * dims[1] <= 4096
    ocs, oci = oracle.cell_list(2, np.float32([0, 0]), np.float32(1.0 / cs_), dims[:2], st.pos[0][:n], st.pos[1][:n],
                                None)
    np.testing.assert_array_equal(cs, ocs)
    counts = np.diff(ocs)
    for m in crowds.values():
        assert (counts >= m).sum() >= 1
    cell_of = np.repeat(np.arange(len(ocs) - 1), counts)
    np.testing.assert_array_equal(ci[np.lexsort((ci, cell_of))], oci[np.lexsort((oci, cell_of))])
    d.close()


# ----------------------------------------------------------- update parity ---

@pytest.mark.parametrize("method", ["counting", "bucketed"])
@pytest.mark.parametrize("name", ["channel2d", "pipe3d_small"])
def test_update_with_each_build_method(name, method, monkeypatch):
    """The merged step's candidates come from the count pass of either build: 40
    steps of each against the oracle (the default automatic choice alternates the
    two while it times them, which every other test goes through)."""
    import tests._gpu as G
    monkeypatch.setattr(G, "BUILD_METHOD", method)
    wl = W.channel2d() if name == "channel2d" else W.pipe3d(dp=0.004)
    g, dl = _run_steps(wl, 40, check_every=10)
    assert g > 0 and dl > 0


def test_automatic_build_method_times_both():
    """SPH_BUILD_AUTO: after a few synchronised builds both methods have been
    timed (positive times, at least the exploration's samples), and the method
    it settles on is the faster one within its 3 % margin."""
    from paper_2406_16786_amd import sphbuf as S
    wl = W.pipe3d(dp=0.004)
    bufs = oracle_buffers(wl)
    d = make_domain(wl, bufs)
    st, m, us, ns = S.sph_build_stats(d.ctx)
    assert st == 0 and m == S.SPH_BUILD_AUTO and ns == [0, 0]
    for _ in range(24):
        d.build()
        d.stream.synchronize()
    st, m, us, ns = S.sph_build_stats(d.ctx)
    assert st == 0 and min(ns) >= 3 and min(us) > 0.0, (us, ns)
    for _ in range(4):
        d.build()
    d.stream.synchronize()
    st, m, us, ns = S.sph_build_stats(d.ctx)
    fast = S.SPH_BUILD_COUNTING if us[0] <= us[1] else S.SPH_BUILD_BUCKETED
    slow = S.SPH_BUILD_BUCKETED if fast == S.SPH_BUILD_COUNTING else S.SPH_BUILD_COUNTING
    assert m == fast or us[slow - 1] * 0.97 <= us[fast - 1] * (1 + 1e-12), (m, us)
    # a retune forgets both times and measures them again
    assert S.sph_build_retune(d.ctx) == 0
    st, m, us, ns = S.sph_build_stats(d.ctx)
    assert st == 0 and ns == [0, 0] and us == [0.0, 0.0]
    for _ in range(12):
        d.build()
        d.stream.synchronize()
    st, m, us, ns = S.sph_build_stats(d.ctx)
    assert st == 0 and min(ns) >= 3 and min(us) > 0.0, (us, ns)
    d.close()


def test_fixed_build_methods_report_themselves():
    """A fixed method runs on every build and is reported as the last build's; no
    timing is taken (both times stay 0)."""
    from paper_2406_16786_amd import sphbuf as S
    import tests._gpu as G
    wl = W.pipe3d(dp=0.004)
    bufs = oracle_buffers(wl)
    for name, code in (("counting", S.SPH_BUILD_COUNTING), ("bucketed", S.SPH_BUILD_BUCKETED)):
        d = G.make_domain_raw(wl.dim, wl.lo, wl.hi, wl.cell_size, wl.dp, bufs, oracle_state(wl), build_method=name)
        for _ in range(3):
            d.build()
        d.stream.synchronize()
        st, m, us, ns = S.sph_build_stats(d.ctx)
        assert st == 0 and m == code and ns == [0, 0] and us == [0.0, 0.0], (name, m, us, ns)
        d.close()


def test_channel2d_200_steps_local():
    g, dl = _run_steps(W.channel2d(), 200)
    assert g > 500 and dl > 300


def test_channel2d_60_steps_fullscan():
    _run_steps(W.channel2d(), 60, mode="fullscan")


@pytest.mark.parametrize("mode", ["local", "fullscan"])
def test_bent_channel_40_steps(mode):
    g, dl = _run_steps(W.bent_channel2d(), 40, mode=mode, check_every=10)
    assert g > 0


def test_bent_channel_1000_steps():
    """The non-orthogonal channel (inlet at +30 deg, outlet at -45 deg, 206 k
    particles) for 1,000 steps of the local-cell path: events every step, every
    array every 100 steps."""
    g, dl = _run_steps(W.bent_channel2d(), 1000, check_every=100)
    assert g > 1000 and dl > 1000


@pytest.mark.parametrize("mode", ["local", "fullscan"])
def test_pipe3d_small_40_steps(mode):
    # dp = 0.004 (about 122k particles): several cells across, ragged tails
    g, dl = _run_steps(W.pipe3d(dp=0.004), 40, mode=mode, check_every=10)
    assert g > 0


def test_pipe3d_small_500_steps():
    """The 3-D pipe scaled to dp = 0.004 (122 k particles) for 500 steps of the
    local-cell path: events every step, every array every 50 steps."""
    g, dl = _run_steps(W.pipe3d(dp=0.004), 500, check_every=50)
    assert g > 1000 and dl > 1000


def test_grid_independence_of_local_path():
    # cell size 1.3 dp and 5.2 dp give the same events as the oracle (no grid)
    wl = W.channel2d()
    for cs in (1.3 * wl.dp, 5.2 * wl.dp):
        _run_steps(wl, 30, cell_size=cs, check_every=10)


# ----------------------------------------------------------- identification ---

def test_identify_each_buffer_separately():
    wl = W.pipe3d(dp=0.004)
    bufs = oracle_buffers(wl)
    st = oracle_state(wl)
    d = make_domain(wl, bufs, st)
    for which in (2, 1):
        rc, nl = oracle.identify(bufs, st, which)
        assert d.identify(which) == 0
        assert_same_state(d, st, f"identify {which}")
    d.close()


# -------------------------------------------------------------- error paths ---

class _Raw:
    """Grid and spacing of a hand-made 2-D case."""
    dim, lo, hi, cell_size, dp = 2, (-1.0, -1.0, 0.0), (6.0, 2.0, 0.0), 0.3, 0.1


def _two_buffer_case(pts, labels, capacity=None):
    bufs = [oracle.Buffer(oracle.INLET, (0.5, 0.5, 0), I3, (0.5, 0.5, 0), 0.25),
            oracle.Buffer(oracle.OUTLET, (4.5, 0.5, 0), I3, (0.5, 0.5, 0), 0.25)]
    st = make_state(2, pts, capacity=capacity, labels=labels, carried=3)
    return _Raw(), bufs, st


def _identify_counts(d, bufs, st):
    # make the library's labelled counts agree with the given labels
    from paper_2406_16786_amd import sphbuf as S
    nl = [int(np.sum(st.label[: st.n] == k + 1)) for k in range(len(bufs))]
    assert S.sph_state_set(d.ctx, st.next_id, nl) == 0


@pytest.mark.parametrize("mode", ["local", "fullscan"])
@pytest.mark.parametrize("case", range(3))
def test_hand_examples_on_gpu(case, mode):
    """tests/golden/hand_examples.json through the library: the hand-worked events,
    layout, ids and carried fields, both update paths."""
    c, bufs, st = golden_cases()[case]
    e = c["expect"]
    dim = c["dim"]
    pts = np.array([p["pos"] for p in c["particles"]])
    lo = [float(pts[:, a].min()) - 1.5 for a in range(dim)] + [0.0] * (3 - dim)
    hi = [float(pts[:, a].max()) + 1.5 for a in range(dim)] + [0.0] * (3 - dim)
    d = make_domain_raw(dim, tuple(lo), tuple(hi), 0.3, 0.1, bufs, st)
    _identify_counts(d, bufs, st)
    if mode == "local":
        d.build()
        gst, g, dl = d.update()
    else:
        gst, g, dl = d.update_fullscan()
    assert gst == 0
    _, gg, dd = d.events()
    assert list(gg) == e["gen"] and list(dd) == e["del"]
    pos, car, lab, ids, n = d.download()
    assert n == e["n"]
    for ax in range(dim):
        np.testing.assert_array_equal(pos[ax][:n], np.float32(e["pos"][ax]))
    assert list(lab[:n]) == e["label"] and list(ids[:n]) == e["id"]
    for f in range(3):
        np.testing.assert_array_equal(car[f][:n], np.float32([10 * s_ + f for s_ in e["source"]]))
    rs, r = d.result()
    assert r.next_id == e["next_id"] and list(r.n_labelled[: len(bufs)]) == e["n_labelled"]
    d.close()


@pytest.mark.parametrize("mode", ["local", "fullscan"])
def test_cfl_violation_leaves_state_untouched(mode):
    pts = [(0.25, 0.5), (1.125, 0.5), (0.7, 0.5)]
    wl, bufs, st = _two_buffer_case(pts, [1, 1, 1])
    d = make_domain(wl, bufs, st)
    _identify_counts(d, bufs, st)
    st.pos[0][2] = np.float32(2.5)      # a buffer particle jumped out of its check region
    upload_state(d, st)
    if mode == "local":
        d.build()
        gst, _, _ = d.update()
    else:
        gst, _, _ = d.update_fullscan()
    assert gst == oracle.update(bufs, st.copy()).status == oracle.ERR_CFL
    assert_same_state(d, st, "cfl")
    d.close()


@pytest.mark.parametrize("mode", ["local", "fullscan"])
def test_capacity_exhaustion_leaves_state_untouched(mode):
    pts = [(1.125, 0.5), (1.2, 0.4), (1.1, 0.3)]
    wl, bufs, st = _two_buffer_case(pts, [1, 1, 1], capacity=4)
    d = make_domain(wl, bufs, st)
    _identify_counts(d, bufs, st)
    if mode == "local":
        d.build()
        gst, _, _ = d.update()
    else:
        gst, _, _ = d.update_fullscan()
    assert gst == oracle.update(bufs, st.copy()).status == oracle.ERR_CAPACITY
    assert_same_state(d, st, "capacity")
    d.close()


@pytest.mark.parametrize("mode", ["local", "fullscan"])
def test_nonfinite_position_leaves_state_untouched(mode):
    pts = [(1.125, 0.5), (np.nan, 0.4), (0.3, 0.3)]
    wl, bufs, st = _two_buffer_case(pts, [1, 0, 1])
    d = make_domain(wl, bufs, st)
    _identify_counts(d, bufs, st)
    if mode == "local":
        d.build()
        gst, _, _ = d.update()
    else:
        gst, _, _ = d.update_fullscan()
    assert gst == oracle.update(bufs, st.copy()).status == oracle.ERR_NONFINITE
    assert_same_state(d, st, "nonfinite")
    d.close()


def test_update_without_build_is_refused():
    from paper_2406_16786_amd import sphbuf as S
    wl, bufs, st = _two_buffer_case([(0.25, 0.5)], [1])
    d = make_domain(wl, bufs, st)
    assert d.update()[0] == S.SPH_ERR_STATE
    d.close()


def test_empty_domain():
    wl, bufs, st = _two_buffer_case(np.zeros((0, 2)), [])
    d = make_domain(wl, bufs, st)
    d.build()
    gst, g, dl = d.update()
    assert (gst, g, dl) == (0, 0, 0)
    d.close()


def test_every_particle_deleted():
    pts = [(5.01 + 0.01 * i, 0.5) for i in range(20)]
    wl, bufs, st = _two_buffer_case(pts, [0] * 20)
    d = make_domain(wl, bufs, st)
    d.build()
    gst, g, dl = d.update()
    res = oracle.update(bufs, st)
    assert gst == 0 and dl == 20 and len(res.dele) == 20 and st.n == 0
    assert_same_state(d, st, "all deleted")
    d.close()


@pytest.mark.parametrize("mode", ["local", "fullscan"])
@pytest.mark.parametrize("n", [200_000, 700_000])
def test_clustered_event_indices(n, mode):
    """Generated sources and deleted particles in long runs of consecutive
    indices plus one far away: with 700k particles a run fills a bucket of the
    finalize's counting sort past its limit (the comparison sort takes over),
    with 200k it does not.  Events and arrays must still equal the oracle's."""
    rng = np.random.default_rng(7)
    pts = np.column_stack([rng.uniform(1.5, 3.5, n), rng.uniform(0.0, 1.0, n)])
    labels = np.zeros(n, np.int32)
    gen = np.r_[np.arange(0, 300), n - 1]
    dele = np.r_[np.arange(1000, 1300), n - 2]
    pts[gen, 0] = rng.uniform(1.01, 1.2, gen.size)     # labelled inlet particles past X' = a/2
    labels[gen] = 1
    pts[dele, 0] = rng.uniform(5.01, 5.2, dele.size)   # past the outlet's X' = a/2
    wl, bufs, st = _two_buffer_case(pts, labels, capacity=n + 400)
    d = make_domain(wl, bufs, st)
    _identify_counts(d, bufs, st)
    if mode == "local":
        d.build()
        gst, g, dl = d.update()
    else:
        gst, g, dl = d.update_fullscan()
    res = oracle.update(bufs, st)
    assert gst == res.status == 0
    np.testing.assert_array_equal(res.gen, gen)
    np.testing.assert_array_equal(res.dele, dele)
    eg, gg, dd = d.events()
    np.testing.assert_array_equal(gg, res.gen)
    np.testing.assert_array_equal(dd, res.dele)
    assert_same_state(d, st, "clustered")
    d.close()


def _misalign(d):
    """Move the domain's coordinate and carried arrays 4 bytes off 16-byte alignment
    (views into one-longer allocations): the kernels must take their scalar paths."""
    import torch
    from paper_2406_16786_amd import sphbuf as S
    for name in ("pos", "carried"):
        views = []
        for t in getattr(d, name):
            big = torch.zeros(t.shape[0] + 1, dtype=t.dtype, device=t.device)
            v = big[1:]
            v.copy_(t)
            views.append(v)
        setattr(d, name, views)
    assert d.pos[0].data_ptr() % 16 != 0
    d.p = S.particles_from_tensors(d.pos, d.carried, d.label, d.id, d.n_dev)


@pytest.mark.parametrize("mode", ["local", "fullscan"])
def test_unaligned_arrays_take_the_scalar_paths(mode):
    wl = W.bent_channel2d()
    bufs = oracle_buffers(wl)
    st = oracle_state(wl)
    d = make_domain(wl, bufs, st)
    _misalign(d)
    assert oracle.identify(bufs, st, -1)[0] == 0 and d.identify(-1) == 0
    for step in range(12):
        W.advect_host(wl, st.pos, st.n, step)
        upload_state(d, st)
        if mode == "local":
            d.build()
            if step == 0:
                cs, ci, dims = _cell_list(d, st.n)
                ocs, oci = oracle.cell_list(2, np.float32(wl.lo[:2]), np.float32(1.0 / wl.cell_size), dims[:2],
                                            st.pos[0][: st.n], st.pos[1][: st.n], None)
                np.testing.assert_array_equal(cs, ocs)
            gst, g, dl = d.update()
        else:
            gst, g, dl = d.update_fullscan()
        res = oracle.update(bufs, st)
        assert gst == res.status == 0
        np.testing.assert_array_equal(d.events()[1], res.gen)
        np.testing.assert_array_equal(d.events()[2], res.dele)
        assert_same_state(d, st, f"step {step}")
    d.close()


def test_checkpoint_and_restore_continue_identically():
    """Library state outside the particle arrays (next id, labelled counts) saved
    mid-run and restored into a fresh context gives the same continuation."""
    from paper_2406_16786_amd import sphbuf as S
    wl = W.bent_channel2d()
    bufs = oracle_buffers(wl)
    st = oracle_state(wl)
    d = make_domain(wl, bufs, st)
    assert d.identify(-1) == 0

    def run(dom, steps, first):
        pos, car, lab, ids, n = dom.download()
        events = []
        for step in range(first, first + steps):
            W.advect_host(wl, pos, n, step)
            dom.upload(pos, car, lab, ids, n)
            dom.build()
            gst, g, dl = dom.update()
            assert gst == 0
            events.append((dom.events()[1].copy(), dom.events()[2].copy()))
            pos, car, lab, ids, n = dom.download()
        return events, (pos, car, lab, ids, n)

    run(d, 10, 0)
    snap = d.download()
    st_, nid, nl = S.sph_state_get(d.ctx)
    assert st_ == 0
    ev1, end1 = run(d, 10, 10)
    pos, car, lab, ids, n = snap
    st2 = oracle.State(wl.dim, [p.copy() for p in pos], [c.copy() for c in car], lab.copy(), ids.copy(), n, nid)
    d2 = make_domain(wl, bufs, st2)
    assert S.sph_state_set(d2.ctx, nid, nl) == 0
    ev2, end2 = run(d2, 10, 10)
    for (g1, d1_), (g2, d2_) in zip(ev1, ev2):
        np.testing.assert_array_equal(g1, g2)
        np.testing.assert_array_equal(d1_, d2_)
    assert end1[4] == end2[4]
    for a1, a2 in zip(end1[0] + end1[1] + [end1[2], end1[3]], end2[0] + end2[1] + [end2[2], end2[3]]):
        np.testing.assert_array_equal(a1[: end1[4]], a2[: end1[4]])
    d.close()
    d2.close()


# ---------------------------------------------------------------- guard band ---

@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("seed", range(3))
def test_guard_band_decisions_equal_fp64(dim, seed):
    """Positions whose FP64 local coordinate lies within 1e-5 dp of a threshold:
    the FP32 pass alone would get some of these wrong, the recheck must not."""
    rng = np.random.default_rng(50 + 10 * dim + seed)
    dp = 0.001
    half = np.array([2 * dp, 0.05, 0.04])
    margin = 2.6 * dp
    if dim == 2:
        q = oracle.rotation_2d(rng.uniform(-math.pi, math.pi))
    else:
        v = rng.standard_normal(3)
        q = oracle.rotation_from_direction(v / np.linalg.norm(v))
    origin = rng.uniform(-1.0, 1.0, 3)
    if dim == 2:
        origin[2] = 0.0
    kinds = [oracle.OUTLET, oracle.BIDIR, oracle.INLET][seed]
    b = oracle.Buffer(kinds, tuple(origin), q, tuple(half), margin)
    n = 10000
    L = rng.uniform(-(half + margin), half + margin, size=(n, 3))
    thr = [half[0], -half[0], half[0] + margin, -(half[0] + margin)]
    c = rng.integers(0, dim, n)
    for i in range(n):   # snap one coordinate next to one of its thresholds
        cc = c[i]
        t = rng.choice([half[cc], -half[cc], half[cc] + margin, -(half[cc] + margin)])
        L[i, cc] = t + rng.uniform(-1e-5, 1e-5) * dp
    if dim == 2:
        L[:, 2] = 0.0
    G = L @ q + origin
    pts = G[:, :dim].astype(np.float32)
    bl = oracle.Buffer(b.kind, b.origin, b.rot, b.half, b.margin)
    st0 = make_state(dim, pts, capacity=2 * n, carried=2)
    lc = local(dim, bl, st0)
    inc = np.all(np.abs(lc[:, :dim]) < (half + margin)[:dim], axis=1)
    labels = ((rng.uniform(size=n) < 0.5) & inc).astype(np.int32)
    st = make_state(dim, pts, capacity=2 * n, labels=labels, carried=2)
    d = make_domain_raw(dim, origin - 0.2, origin + 0.2, 2.6 * dp, dp, [bl], st, max_events=4096)
    from paper_2406_16786_amd import sphbuf as S
    assert S.sph_state_set(d.ctx, st.next_id, [int(labels.sum())]) == 0
    d.build()
    gst, g, dl = d.update()
    res = oracle.update([bl], st)
    assert gst == res.status == 0
    eg, gg, dd = d.events()
    np.testing.assert_array_equal(gg, res.gen)
    np.testing.assert_array_equal(dd, res.dele)
    assert_same_state(d, st, "guard band")
    d.close()


# --------------------------------------------------------- determinism ---

def test_repeat_runs_are_identical():
    wl = W.bent_channel2d()
    outs = []
    for _ in range(2):
        bufs = oracle_buffers(wl)
        st = oracle_state(wl)
        d = make_domain(wl, bufs, st)
        d.identify(-1)
        for step in range(5):
            pos, car, lab, ids, n = d.download()
            W.advect_host(wl, pos, n, step)
            d.upload(pos, car, lab, ids, n)
            d.build()
            assert d.update()[0] == 0
        outs.append(d.download())
        d.close()
    a, b = outs
    for x, y in zip(a[0] + a[1] + [a[2], a[3]], b[0] + b[1] + [b[2], b[3]]):
        np.testing.assert_array_equal(x, y)


# ------------------------------------------------------------ full size ---

@pytest.mark.parametrize("mode", ["local", "fullscan"])
def test_pipe3d_full_size_three_steps(mode):
    """The 3-D pipe at dp = 0.001 (7.86 M particles), the size the benchmark
    times: events and every array against the oracle for three updates."""
    _run_steps(W.pipe3d(), 3, mode=mode)


# -------------------------------------------- bidirectional tree, sparse grid ---

def test_celllist_sparse_matches_oracle():
    wl = W.tree3d(dp=0.004)
    bufs = oracle_buffers(wl)
    d = make_domain(wl, bufs, brick_log2=3, brick_margin=1)
    d.build()
    cs, ci, dims = _cell_list(d, wl.n)
    lo32 = np.float32(wl.lo[:3])
    inv = np.float32(1.0 / wl.cell_size)
    x, y, z = wl.pos[0][: wl.n], wl.pos[1][: wl.n], wl.pos[2][: wl.n]
    act = oracle.sparse_active(3, lo32, inv, dims, 3, 1, x, y, z)
    ocs, oci = oracle.cell_list_sparse(3, lo32, inv, dims, 3, act, x, y, z)
    np.testing.assert_array_equal(cs, ocs)
    cell_of = np.repeat(np.arange(len(ocs) - 1), np.diff(ocs))
    np.testing.assert_array_equal(ci[np.lexsort((ci, cell_of))], oci)
    d.close()


@pytest.mark.parametrize("mode", ["local", "fullscan"])
def test_tree_bidirectional_one_period(mode):
    """Branching pipe network, dp = 0.004 (about 250k particles), four
    bidirectional buffers, one full period of the reversing flow: every buffer
    generates and deletes; brick-sparse grid for the local path."""
    wl = W.tree3d(dp=0.004)
    g, dl = _run_steps(wl, 200, mode=mode, check_every=25, brick_log2=3)
    assert g > 100 and dl > 100


def test_tree_full_size_two_steps():
    """The branching network at dp = 0.001 (about 16 M particles) on the
    brick-sparse grid: events and every array against the oracle."""
    _run_steps(W.tree3d(), 2, mode="local", brick_log2=3)


@pytest.mark.parametrize("path", ["merged", "cells", "fullscan"])
def test_far_wide_grid_fp32_binning(path):
    """A 2-D grid of 150,000 cells along x whose origin is 10^6 cells from 0 (FP32
    binning is off by up to ~0.07 cells): an axis-aligned outlet whose check region
    starts just left of an FP32 column that bins a cell too low, with buffer
    particles on that column (they must be found, relabelled to fluid, and counted
    by the CFL check), plus an oblique outlet with a few thousand particles near
    the boundary of its check region.  Events and arrays equal the oracle's."""
    import math
    from tests.test_abi_host import WIDE_CS, WIDE_DIMS, WIDE_DP, WIDE_LO, misbinned_column
    cs, dp, lo, dims = WIDE_CS, WIDE_DP, WIDE_LO, WIDE_DIMS
    half = np.array([2 * dp, 0.012, 0.0])
    ext = (half + cs)[:2]
    xc, k = misbinned_column(lo, cs, dims, dims[0] - 300)
    o1 = np.array([xc - 1e-9 + ext[0], 0.0012, 0.0])
    q2 = oracle.rotation_2d(math.radians(-35.0))
    o2 = np.array([lo[0] + (dims[0] - 40) * cs, 0.0012, 0.0])
    bufs = [oracle.Buffer(oracle.OUTLET, tuple(o1), np.eye(3), tuple(half), cs),
            oracle.Buffer(oracle.OUTLET, tuple(o2), q2, tuple(half), cs)]
    rng = np.random.default_rng(21)
    col = np.column_stack([np.full(60, np.float32(xc)), np.linspace(o1[1] - 0.9 * ext[1], o1[1] + 0.9 * ext[1], 60)])
    box1 = np.column_stack([rng.uniform(o1[0] - half[0], o1[0] + half[0], 200),
                            rng.uniform(o1[1] - half[1], o1[1] + half[1], 200)])
    L = rng.uniform(-1.05, 1.05, size=(3000, 2)) * ext
    side = rng.integers(0, 2, 3000)
    L[np.arange(3000), side] = np.sign(L[np.arange(3000), side]) * ext[side] * rng.uniform(0.9, 1.02, 3000)
    obl = L @ q2[:2, :2] + o2[:2]
    pts = np.concatenate([col, box1, obl]).astype(np.float32).astype(np.float64)
    labels = np.zeros(len(pts), np.int32)
    labels[:60] = 1                                  # buffer particles of outlet 1 in its margin
    labels[60:260] = 1                               # ... and in its box
    lc2 = oracle.local_coords(2, bufs[1], pts[:, 0].astype(np.float32), pts[:, 1].astype(np.float32), None)
    in_box2 = np.all(np.abs(lc2[:, :2]) < half[:2], axis=1)
    labels[260:][in_box2[260:]] = 2
    st = make_state(2, pts, capacity=len(pts) + 64, labels=labels)
    hi = lo + (np.array(dims) - 0.5) * cs
    d = make_domain_raw(2, tuple(lo), tuple(hi), cs, dp, bufs, st,
                        update_path="cells" if path == "cells" else "merged")
    _identify_counts(d, bufs, st)
    if path == "fullscan":
        gst, g, dl = d.update_fullscan()
    else:
        d.build()
        gst, g, dl = d.update()
    res = oracle.update(bufs, st)
    assert gst == res.status == 0, (gst, res.status)
    _, gg, dd = d.events()
    np.testing.assert_array_equal(gg, res.gen)
    np.testing.assert_array_equal(dd, res.dele)
    assert len(res.dele) > 0
    assert_same_state(d, st, "far wide grid")
    assert np.all(st.label[:60] == 0)                # the column's buffer particles were relabelled
    d.close()
