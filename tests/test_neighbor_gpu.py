"""GPU parity of the neighbour search over the library's cell list (the solver's
reuse of it; kernel support 2h of Section 3 = the cell size) against the oracle's
brute force over all particles: counts identical, particle by particle."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests._gpu import make_domain, make_domain_raw, upload_state
from tests._support import make_state, oracle_buffers, oracle_state

pytestmark = pytest.mark.gpu


def _S():
    from paper_2406_16786_amd import sphbuf as S
    return S


def _gpu_counts(d, radius):
    st, counts = d.neighbor_count(radius)
    assert st == 0, st
    return counts.cpu().numpy()


def _oracle_counts(st, radius, query=None):
    n = st.n
    z = st.pos[2][:n] if st.dim == 3 else None
    return oracle.neighbor_count(st.dim, st.pos[0][:n], st.pos[1][:n], z, radius, query)


def test_channel2d_every_particle():
    wl = W.channel2d()
    bufs = oracle_buffers(wl)
    st = oracle_state(wl)
    d = make_domain(wl, bufs, st)
    d.build()
    for radius in (wl.cell_size, 0.5 * wl.cell_size, 1.01 * wl.dp):
        c = _gpu_counts(d, radius)
        np.testing.assert_array_equal(c[: st.n], _oracle_counts(st, radius), err_msg=f"radius {radius}")
        assert np.all(c[st.n:] == -1)  # entries past N are left alone
    d.close()


def test_pipe3d_small_sampled():
    wl = W.pipe3d(dp=0.004)
    bufs = oracle_buffers(wl)
    st = oracle_state(wl)
    d = make_domain(wl, bufs, st)
    d.build()
    c = _gpu_counts(d, wl.cell_size)
    rng = np.random.Generator(np.random.PCG64(3))
    q = np.unique(np.concatenate([rng.choice(st.n, 3000, replace=False), [0, st.n - 1]]))
    np.testing.assert_array_equal(c[q], _oracle_counts(st, wl.cell_size, q))
    d.close()


def test_brick_sparse_grid_with_particles_in_inactive_bricks():
    wl = W.hub_domain(1, 20000, 3, 3)
    bufs = oracle_buffers(wl)
    st = oracle_state(wl)
    d = make_domain(wl, bufs, st, brick_log2=3)   # fits the active bricks to these positions
    # move 40 particles into a cluster in a corner of the box, far from the fluid:
    # their bricks are inactive, so they share the overflow cell
    rng = np.random.Generator(np.random.PCG64(8))
    moved = rng.choice(st.n, 40, replace=False)
    corner = np.array(wl.lo[:3]) + 2.0 * wl.cell_size
    for c in range(3):
        st.pos[c][moved] = (corner[c] + rng.uniform(0.0, 1.5 * wl.cell_size, moved.size)).astype(np.float32)
    upload_state(d, st)
    d.build()
    c = _gpu_counts(d, wl.cell_size)
    np.testing.assert_array_equal(c[: st.n], _oracle_counts(st, wl.cell_size))
    assert c[moved].min() > 0
    d.close()


def test_particles_outside_the_grid_and_nan():
    rng = np.random.Generator(np.random.PCG64(5))
    pts = rng.uniform(-0.3, 1.3, size=(3000, 2))        # the grid covers [0, 1]^2
    pts[17] = np.nan
    st = make_state(2, pts)
    d = make_domain_raw(2, (0.0, 0.0, 0.0), (1.0, 1.0, 0.0), 0.05, 0.02, [], st)
    d.build()
    c = _gpu_counts(d, 0.05)
    np.testing.assert_array_equal(c[: st.n], _oracle_counts(st, 0.05))
    assert c[17] == 0
    d.close()


def _face_pairs(lo: float, cs: float, kmax: int, count: int):
    """Pairs (x_i, x_j) on one axis, less than one cell apart, whose FP32 cell
    coordinates floor(fl(fl(x - lo) * fl(1 / cs))) differ by two (the rounding of
    the subtraction and of the product going opposite ways near two faces)."""
    lo32, inv = np.float32(lo), np.float32(1.0 / cs)

    def cell(x):
        return int(np.floor(np.float32(np.float32(x - lo32) * inv)))

    def around(x0):
        xs, a, b = [x0], x0, x0
        for _ in range(16):
            a = np.nextafter(a, np.float32(-np.inf))
            b = np.nextafter(b, np.float32(np.inf))
            xs += [a, b]
        return xs

    out = []
    for k in range(kmax // 4, kmax - 3):
        ci = [x for x in around(np.float32(float(lo32) + (k + 1) * cs)) if cell(x) == k]
        cj = [x for x in around(np.float32(float(lo32) + (k + 2) * cs)) if cell(x) == k + 2]
        if ci and cj and float(min(cj)) - float(max(ci)) < cs:
            out.append((max(ci), min(cj)))
            if len(out) >= count:
                break
    return out


def test_pairs_two_fp32_cells_apart_are_found():
    cs, dims, lo = 0.0026, 3000, -3.1
    pairs = _face_pairs(lo, cs, dims, 24)
    assert len(pairs) >= 8, "no FP32 binning pair two cells apart found"
    pts = []
    for r, (xi, xj) in enumerate(pairs):
        y = 0.01 + 3.0 * r * cs                      # rows far apart
        pts += [(float(xi), y), (float(xj), y)]
    st = make_state(2, np.array(pts))
    d = make_domain_raw(2, (lo, 0.0, 0.0), (lo + dims * cs, 1.0, 0.0), cs, cs / 2.6, [], st)
    d.build()
    c = _gpu_counts(d, cs)
    ref = _oracle_counts(st, cs)
    np.testing.assert_array_equal(c[: st.n], ref)
    assert np.all(ref == 1)
    d.close()


def test_empty_domain():
    st = make_state(3, np.zeros((0, 3)))
    d = make_domain_raw(3, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 0.1, 0.04, [], st)
    d.build()
    c = _gpu_counts(d, 0.1)
    assert np.all(c == -1)
    d.close()


def test_neighbor_count_arguments_and_state():
    S = _S()
    wl = W.channel2d()
    bufs = oracle_buffers(wl)
    st = oracle_state(wl)
    d = make_domain(wl, bufs, st)
    assert d.neighbor_count(wl.cell_size)[0] == S.SPH_ERR_STATE        # no cell list yet
    d.build()
    for r in (0.0, -1.0, 1.0001 * wl.cell_size, float("nan")):
        assert d.neighbor_count(r)[0] == S.SPH_ERR_ARG, r
    assert d.neighbor_count(wl.cell_size)[0] == 0
    assert d.identify(-1) == 0
    d.build()
    assert d.update()[0] == 0
    assert d.neighbor_count(wl.cell_size)[0] == S.SPH_ERR_STATE        # positions changed since the build
    d.close()


def test_pipe3d_full_size_sampled():
    wl = W.pipe3d()
    bufs = oracle_buffers(wl)
    st = oracle_state(wl)
    d = make_domain(wl, bufs, st)
    d.build()
    c = _gpu_counts(d, wl.cell_size)
    rng = np.random.Generator(np.random.PCG64(4))
    q = rng.choice(st.n, 120, replace=False)
    np.testing.assert_array_equal(c[q], _oracle_counts(st, wl.cell_size, q))
    d.close()
