"""Pins for the FP64 oracle: facts fixed by the paper or by mathematics, checked
without trusting the oracle's own formulas.

 * closed forms of the frames (Eq. 2D_transformation, Eqs. rotation_axis to
   3D_transformation, Eq. rotation_matrix against scipy's rotation vectors);
 * hand-worked updates whose expected events and final arrays are written out
   by reasoning from Algorithms 1-3 (inlet, outlet, bidirectional, 3-D frame);
 * the axis-aligned special case, where every test is a plain interval check
   (the textbook orthogonal buffer of the introduction);
 * rotation invariance: the same local configuration placed with and without a
   rotation gives the same events;
 * balances and invariants over a 200-step run of the 2-D channel;
 * the steady inflow rate (particles per step = flux * dt / dp^2);
 * strict thresholds, error paths leaving the state untouched.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import workloads as W
from tests._support import golden_cases, local, make_state, oracle_buffers, oracle_state

I3 = np.eye(3)


# --------------------------------------------------------------- frames ---

def test_rotation_2d_quarter_turn_closed_form():
    # Eq. (2D_transformation) with theta = 90 deg, O' = 0: X' = Y, Y' = -X.
    q = oracle.rotation_2d(math.pi / 2)
    b = oracle.Buffer(oracle.INLET, (0, 0, 0), q, (1, 1, 1), 0.1)
    lc = oracle.local_coords(2, b, np.float32([3.0, -2.0]), np.float32([5.0, 7.0]))
    np.testing.assert_allclose(lc[:, 0], [5.0, 7.0], atol=1e-15)
    np.testing.assert_allclose(lc[:, 1], [-3.0, 2.0], atol=1e-15)


def test_rotation_2d_thirty_degrees_by_hand():
    q = oracle.rotation_2d(math.radians(30.0))
    c, s = math.sqrt(3.0) / 2.0, 0.5
    np.testing.assert_allclose(q, [[c, s, 0], [-s, c, 0], [0, 0, 1]], atol=1e-16)
    # inflow normal u = M^T e_x = (cos, sin) (Eq. 2D_normal_transformation)
    np.testing.assert_allclose(q.T @ [1, 0, 0], [c, s, 0], atol=1e-16)


@pytest.mark.parametrize("seed", range(8))
def test_rodrigues_matches_scipy_rotation_vector(seed):
    # Eq. (rotation_matrix) is the active rotation by theta about n.
    rng = np.random.default_rng(seed)
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    th = rng.uniform(0.0, math.pi)
    ref = Rotation.from_rotvec(n * th).as_matrix()
    np.testing.assert_allclose(oracle.rodrigues(n, th), ref, atol=1e-14)


@pytest.mark.parametrize("seed", range(16))
def test_rotation_from_direction_properties(seed):
    rng = np.random.default_rng(100 + seed)
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    q = oracle.rotation_from_direction(d)
    np.testing.assert_allclose(q @ d, [1, 0, 0], atol=1e-14)          # X' along d
    np.testing.assert_allclose(q @ q.T, I3, atol=1e-14)
    assert abs(np.linalg.det(q) - 1.0) < 1e-14
    # the rotation axis e_x x d is left fixed (minimal rotation)
    n = np.cross([1, 0, 0], d)
    n /= np.linalg.norm(n)
    np.testing.assert_allclose(q @ n, n, atol=1e-14)


@pytest.mark.parametrize("deg", [-170, -135, -45, -10, 10, 30, 90, 150, 179])
def test_rotation_from_direction_reduces_to_2d_matrix(deg):
    t = math.radians(deg)
    q3 = oracle.rotation_from_direction([math.cos(t), math.sin(t), 0.0])
    np.testing.assert_allclose(q3, oracle.rotation_2d(t), atol=1e-15)


def test_rotation_from_direction_degenerate_axes():
    np.testing.assert_array_equal(oracle.rotation_from_direction([2.0, 0, 0]), I3)
    np.testing.assert_array_equal(oracle.rotation_from_direction([-1.0, 0, 0]), np.diag([-1.0, -1.0, 1.0]))
    with pytest.raises(ValueError):
        oracle.rotation_from_direction([0.0, 0.0, 0.0])


def test_rotation_from_direction_z_axis_by_hand():
    # d = e_z: n = e_x x e_z / |.| = -e_y, theta = 90 deg.  R rotates e_x->e_z,
    # e_y->e_y, e_z->-e_x, so Q = R^T has rows (e_z, e_y, -e_x).
    q = oracle.rotation_from_direction([0, 0, 1])
    np.testing.assert_allclose(q, [[0, 0, 1], [0, 1, 0], [-1, 0, 0]], atol=1e-15)


def test_local_coords_identity_frame_is_translation():
    b = oracle.Buffer(oracle.INLET, (1.0, 2.0, 3.0), I3, (1, 1, 1), 0.1)
    x, y, z = np.float32([1.5, -4.0]), np.float32([2.25, 0.0]), np.float32([3.0, 8.0])
    lc = oracle.local_coords(3, b, x, y, z)
    np.testing.assert_array_equal(lc, [[0.5, 0.25, 0.0], [-5.0, -2.0, 5.0]])


@pytest.mark.parametrize("seed", range(6))
def test_literal_inverse_transform_equals_shift_along_direction(seed):
    # Eq. (3D_Inverse_transformation): Q^T (Q (r - O') - [a,0,0]) + O' == r - a d.
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    q = oracle.rotation_from_direction(d)
    b = oracle.Buffer(oracle.INLET, tuple(rng.uniform(-3, 3, 3)), q, (0.004, 0.05, 0.05), 0.0026)
    for _ in range(20):
        r = rng.uniform(-3, 3, 3)
        np.testing.assert_allclose(oracle.recycle_literal(3, b, r), r - 0.008 * d, rtol=0, atol=1e-12 * 3)


# ------------------------------------------------ hand-worked updates ---

def _inlet_outlet_2d():
    inlet = oracle.Buffer(oracle.INLET, (0.5, 0.5, 0), I3, (0.5, 0.5, 0), 0.25)
    outlet = oracle.Buffer(oracle.OUTLET, (4.5, 0.5, 0), I3, (0.5, 0.5, 0), 0.25)
    return [inlet, outlet]


@pytest.mark.parametrize("case", range(3))
def test_hand_examples(case):
    """tests/golden/hand_examples.json: three updates worked out by hand (an inlet and
    an outlet in 2-D, a bidirectional buffer under a quarter turn, a 3-D frame along
    e_z), every particle's fate, layout and id against the oracle."""
    c, bufs, st = golden_cases()[case]
    e = c["expect"]
    res = oracle.update(bufs, st)
    assert res.status == oracle.OK
    assert list(res.gen) == e["gen"] and list(res.dele) == e["del"]
    assert st.n == e["n"] and st.next_id == e["next_id"]
    n = st.n
    for ax in range(c["dim"]):
        np.testing.assert_array_equal(st.pos[ax][:n], np.float32(e["pos"][ax]))
    assert list(st.label[:n]) == e["label"]
    assert list(st.id[:n]) == e["id"]
    for f in range(3):
        np.testing.assert_array_equal(st.carried[f][:n], np.float32([10 * s_ + f for s_ in e["source"]]))
    assert list(res.n_labelled) == e["n_labelled"]


def test_identification_labels_box_particles_only():
    bufs = _inlet_outlet_2d()
    st = make_state(2, [(0.5, 0.5), (1.0, 0.5), (-0.1, 0.5), (4.5, 0.99), (4.5, 1.01)])
    rc, nl = oracle.identify(bufs, st, -1)
    assert rc == oracle.OK
    assert list(st.label[:5]) == [1, 0, 0, 2, 0]   # x = 1.0 is on the face: not strictly inside
    assert list(nl) == [1, 1]
    st2 = make_state(2, [(0.5, 0.5), (4.5, 0.5)])
    rc, nl = oracle.identify(bufs, st2, 2)
    assert list(st2.label[:2]) == [0, 2]


def test_threshold_is_strict():
    b = [oracle.Buffer(oracle.OUTLET, (0, 0, 0), I3, (0.5, 0.5, 0), 0.25)]
    on = np.float32(0.5)
    above = np.nextafter(on, np.float32(1))
    st = make_state(2, [(on, 0.0), (above, 0.0)])
    res = oracle.update(b, st)
    assert list(res.dele) == [1]


# ------------------------------------------------------ error paths ---

def _snapshot(st):
    return [a.copy() for a in st.pos + st.carried + [st.label, st.id]], st.n, st.next_id


def _unchanged(st, snap):
    arrs, n, nid = snap
    for a, b in zip(st.pos + st.carried + [st.label, st.id], arrs):
        np.testing.assert_array_equal(a, b)
    assert st.n == n and st.next_id == nid


def test_cfl_violation_is_an_error_without_mutation():
    q = oracle.rotation_from_direction([0, 0, 1])
    b = oracle.Buffer(oracle.INLET, (0, 0, 0), q, (0.5, 1.0, 2.0), 0.25)
    st = make_state(3, [(0.0, 0.0, 0.625), (0.0, 1.5, 0.0)], labels=[1, 1])
    snap = _snapshot(st)
    assert oracle.update([b], st).status == oracle.ERR_CFL
    _unchanged(st, snap)


def test_capacity_exhaustion_is_an_error_without_mutation():
    st = make_state(2, [(1.125, 0.5), (1.2, 0.4), (1.1, 0.3)], capacity=4, labels=[1, 1, 1])
    snap = _snapshot(st)
    assert oracle.update(_inlet_outlet_2d(), st).status == oracle.ERR_CAPACITY
    _unchanged(st, snap)


def test_nonfinite_position_is_an_error_without_mutation():
    st = make_state(2, [(1.125, 0.5), (np.nan, 0.4)], labels=[1, 0])
    snap = _snapshot(st)
    assert oracle.update(_inlet_outlet_2d(), st).status == oracle.ERR_NONFINITE
    _unchanged(st, snap)


# ------------------------------------------- axis-aligned special case ---

def _interval_events(pts, labels, bufs, dim):
    """Events of axis-aligned buffers by interval tests only (no frames)."""
    gen, dele = [], []
    for i, p in enumerate(pts):
        for k, b in enumerate(bufs):
            lo_c = [b.origin[c] - b.half[c] - b.margin for c in range(dim)]
            hi_c = [b.origin[c] + b.half[c] + b.margin for c in range(dim)]
            if not all(lo_c[c] < float(p[c]) < hi_c[c] for c in range(dim)):
                continue
            front = float(p[0]) > b.origin[0] + b.half[0]
            back = float(p[0]) < b.origin[0] - b.half[0]
            mine = labels[i] == k + 1
            if b.kind == oracle.INLET and mine and front:
                gen.append(i)
            elif b.kind == oracle.OUTLET and front:
                dele.append(i)
            elif b.kind == oracle.BIDIR and mine and front:
                gen.append(i)
            elif b.kind == oracle.BIDIR and mine and back:
                dele.append(i)
    return gen, dele


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("seed", range(4))
def test_axis_aligned_buffers_reduce_to_interval_tests(dim, seed):
    rng = np.random.default_rng(seed)
    # dyadic origins/extents so every interval bound is exact in FP64
    bufs = [oracle.Buffer(oracle.INLET, (0.25, 0.5, 0.5), I3, (0.25, 0.5, 0.5), 0.125),
            oracle.Buffer(oracle.OUTLET, (3.0, 0.5, 0.5), I3, (0.25, 0.5, 0.5), 0.125),
            oracle.Buffer(oracle.BIDIR, (1.75, 2.5, 0.5), I3, (0.25, 0.5, 0.5), 0.125)]
    n = 3000
    pts = np.stack([rng.uniform(-0.2, 3.5, n), rng.uniform(-0.2, 3.2, n), rng.uniform(-0.2, 1.2, n)], 1)
    pts = pts[:, :dim].astype(np.float32)
    labels = np.zeros(n, np.int32)
    st0 = make_state(dim, pts, capacity=2 * n)
    oracle.identify(bufs, st0, -1)
    labels[:] = st0.label[:n]
    # move the labelled ones a little so some cross; keep every mover in its region
    pts2 = pts.copy()
    for k, b in enumerate(bufs):
        sel = labels == k + 1
        reach = 0.999 * (b.half[0] + b.margin)
        pts2[sel, 0] = (b.origin[0] + rng.uniform(-reach, reach, int(sel.sum()))).astype(np.float32)
    st = make_state(dim, pts2, capacity=2 * n, labels=labels)
    exp_gen, exp_del = _interval_events(pts2, labels, bufs, dim)
    res = oracle.update(bufs, st)
    assert res.status == oracle.OK
    assert list(res.gen) == exp_gen and list(res.dele) == exp_del
    assert len(exp_gen) > 0 and len(exp_del) > 0


# ----------------------------------------------- rotation invariance ---

@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kind", [oracle.INLET, oracle.OUTLET, oracle.BIDIR])
@pytest.mark.parametrize("seed", range(3))
def test_rotation_invariance(dim, kind, seed):
    rng = np.random.default_rng(1000 * dim + 10 * kind + seed)
    half = np.array([0.004, 0.05, 0.03])
    margin = 0.0026
    n = 4000
    lim = half + 2 * margin
    L = rng.uniform(-lim, lim, size=(n, 3))
    if dim == 2:
        L[:, 2] = 0.0
    # keep points away from every threshold so FP32 placement cannot flip a test
    ok = np.ones(n, bool)
    for c in range(dim):
        for t in (half[c], half[c] + margin):
            ok &= np.abs(np.abs(L[:, c]) - t) > 2e-5
    L = L[ok]
    n = L.shape[0]
    in_check = np.all(np.abs(L[:, :dim]) < (half + margin)[:dim], axis=1)
    labels = ((rng.uniform(size=n) < 0.5) & in_check).astype(np.int32)
    if dim == 2:
        theta = rng.uniform(-math.pi, math.pi)
        q = oracle.rotation_2d(theta)
    else:
        d = rng.standard_normal(3)
        q = oracle.rotation_from_direction(d / np.linalg.norm(d))
    origin = rng.uniform(-1.0, 1.0, 3)
    if dim == 2:
        origin[2] = 0.0
    G = L @ q + origin                    # r = Q^T r' + O'
    ref = oracle.Buffer(kind, (0, 0, 0), I3, tuple(half), margin)
    rot = oracle.Buffer(kind, tuple(origin), q, tuple(half), margin)
    s_ref = make_state(dim, L[:, :dim], capacity=2 * n, labels=labels)
    s_rot = make_state(dim, G[:, :dim], capacity=2 * n, labels=labels)
    r1 = oracle.update([ref], s_ref)
    r2 = oracle.update([rot], s_rot)
    assert r1.status == r2.status == oracle.OK
    np.testing.assert_array_equal(r1.gen, r2.gen)
    np.testing.assert_array_equal(r1.dele, r2.dele)
    np.testing.assert_array_equal(s_ref.label[: s_ref.n], s_rot.label[: s_rot.n])
    assert len(r1.gen) + len(r1.dele) > 0


# ------------------------------------- multi-step balances (2-D channel) ---

def test_channel2d_balances_over_200_steps():
    wl = W.channel2d()
    bufs = oracle_buffers(wl)
    st = oracle_state(wl)
    rc, nl0 = oracle.identify(bufs, st, 1)
    assert rc == oracle.OK and nl0[0] == 80           # 4 columns x 20 rows
    mass_idx = wl.dim
    gens = []
    for step in range(wl.steps):
        W.advect_host(wl, st.pos, st.n, step)
        pre = st.copy()
        lc_pre = [local(2, b, pre) for b in bufs]
        n0 = st.n
        m0 = float(np.sum(st.carried[mass_idx][:n0], dtype=np.float64))
        res = oracle.update(bufs, st)
        assert res.status == oracle.OK
        g, d = res.gen, res.dele
        gens.append(len(g))
        # particle-count and mass balance
        assert st.n == n0 - len(d) + len(g)
        m_del = float(np.sum(pre.carried[mass_idx][d], dtype=np.float64))
        m_gen = float(np.sum(pre.carried[mass_idx][g], dtype=np.float64))
        m1 = float(np.sum(st.carried[mass_idx][: st.n], dtype=np.float64))
        assert abs(m1 - (m0 - m_del + m_gen)) < 1e-9
        # the inlet's buffer set never changes size
        assert res.n_labelled[0] == 80
        # duplicates: pre-recycle state of their sources, label 0, fresh ids
        np0 = n0 - len(d)
        for j, src in enumerate(g):
            for c in range(2):
                assert st.pos[c][np0 + j] == pre.pos[c][src]
            for f in range(len(st.carried)):
                assert st.carried[f][np0 + j] == pre.carried[f][src]
            assert st.label[np0 + j] == 0 and st.id[np0 + j] == pre.next_id + j
        # recycled: X' moved back by exactly one buffer length (FP32 storage)
        ids_after = {int(v): i for i, v in enumerate(st.id[: st.n])}
        for src in g:
            i_new = ids_after[int(pre.id[src])]
            x_new = float(st.pos[0][i_new])
            assert abs((x_new - bufs[0].origin[0]) - (lc_pre[0][src, 0] - 0.08)) < 1e-7
        # ids stay unique, and every labelled particle lies in its check region
        assert len(ids_after) == st.n
        for k, b in enumerate(bufs):
            lc = local(2, b, st)
            sel = st.label[: st.n] == k + 1
            assert np.all(np.abs(lc[sel, 0]) < b.half[0] + b.margin)
    # steady inflow: u = 1, height 0.4, dp = 0.02, dt = 0.005 -> 1 * 0.4 / dp^2 * dt = 5 per step
    assert 4.5 < np.mean(gens[20:]) < 5.5


# -------------------------------------------------------------- cell lists ---

@pytest.mark.parametrize("dim", [2, 3])
def test_cell_list_properties(dim):
    """Counting sort: a permutation, ascending within each cell, and every
    particle's cell box (exact FP64 geometry) contains it unless it lies within
    1e-4 of a cell of a face, where FP32 binning may pick the neighbour."""
    rng = np.random.default_rng(dim)
    n = 5000
    lo, cs = np.array([-0.3, -0.2, -0.1]), 0.05
    dims = [16, 12, 9]
    P = rng.uniform(lo, lo + np.array(dims) * cs, size=(n, 3)).astype(np.float32)
    start, idx = oracle.cell_list(dim, np.float32(lo[:dim]), np.float32(1 / cs), dims[:dim], P[:, 0], P[:, 1],
                                  P[:, 2] if dim == 3 else None)
    assert start[0] == 0 and start[-1] == n and np.all(np.diff(start) >= 0)
    assert np.array_equal(np.sort(idx), np.arange(n))
    C = len(start) - 1
    for c in range(C):
        members = idx[start[c]:start[c + 1]]
        assert np.all(np.diff(members) > 0)
        ix = c % dims[0]
        iy = (c // dims[0]) % dims[1]
        iz = c // (dims[0] * dims[1])
        for i in members:
            for a, k in zip(range(dim), (ix, iy, iz)):
                t = (float(P[i, a]) - lo[a]) / cs
                assert k - 1e-4 < t < k + 1 + 1e-4


def test_cell_list_clamps_outsiders_to_edge_cells():
    start, idx = oracle.cell_list(2, np.float32([0, 0]), np.float32(1.0), [4, 4], np.float32([-5.0, 9.5, 1.5]),
                                  np.float32([1.5, 1.5, 99.0]))
    # cells: (-5, 1.5) -> (0, 1) = 4; (9.5, 1.5) -> (3, 1) = 7; (1.5, 99) -> (1, 3) = 13
    assert list(np.repeat(np.arange(16), np.diff(start))[np.argsort(idx)]) == [4, 7, 13]


def test_sparse_grid_hand_example():
    # 16 x 16 cells of size 1, bricks of 4 x 4 cells (4 x 4 bricks)
    lo, inv, dims = np.float32([0, 0]), np.float32(1.0), [16, 16]
    x = np.float32([5.5, 13.5])   # cells (5, 5) in brick (1, 1) and (13, 2) in brick (3, 0)
    y = np.float32([5.5, 2.5])
    act0 = oracle.sparse_active(2, lo, inv, dims, 2, 0, x, y)
    assert list(np.nonzero(act0)[0]) == [3, 5]          # bricks 3 + 4 * 0 and 1 + 4 * 1
    start, idx = oracle.cell_list_sparse(2, lo, inv, dims, 2, act0, x, y)
    keys = np.repeat(np.arange(len(start) - 1), np.diff(start))[np.argsort(idx)]
    # brick 3 -> slot 0: key 0 * 16 + 1 + 4 * 2 = 9; brick 5 -> slot 1: 16 + 1 + 4 * 1 = 21
    assert list(keys) == [21, 9] and len(start) == 2 * 16 + 2
    act1 = oracle.sparse_active(2, lo, inv, dims, 2, 1, x, y)
    assert int(act1.sum()) == 11                         # 3 x 3 around (1,1) plus 2 x 2 at (2..3, 0..1), 2 shared
    # a particle in an inactive brick goes to the overflow key (last)
    x2, y2 = np.float32([5.5, 13.5, 15.5]), np.float32([5.5, 2.5, 15.5])
    s2, i2 = oracle.cell_list_sparse(2, lo, inv, dims, 2, act0, x2, y2)
    keys2 = np.repeat(np.arange(len(s2) - 1), np.diff(s2))[np.argsort(i2)]
    assert list(keys2) == [21, 9, 32]
