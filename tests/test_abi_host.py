"""CPU tests of the C-ABI library: it loads, exports every declared symbol, and its
host-side FP64 helpers (frames, validation, cell cover, guard band) behave as
specified.  No kernel is launched here."""
import math
import re
import os

import numpy as np
import pytest

import oracle
from paper_2406_16786_amd import sphbuf as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sphbuf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = S.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(S.EXPORTED) == names


def test_status_strings():
    for s in range(11):
        assert S.sph_status_str(s) and S.sph_status_str(s) != "unknown status"


@pytest.mark.parametrize("deg", [-170, -45, 0, 30, 90, 135])
def test_rotation_2d_matches_oracle(deg):
    st, q = S.sph_rotation_2d(math.radians(deg))
    assert st == 0
    np.testing.assert_allclose(q, oracle.rotation_2d(math.radians(deg)), atol=1e-16)


@pytest.mark.parametrize("seed", range(10))
def test_rotation_from_direction_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(3)
    st, q = S.sph_rotation_from_direction(d)
    assert st == 0
    np.testing.assert_allclose(q, oracle.rotation_from_direction(d), atol=1e-15)
    np.testing.assert_allclose(q @ (d / np.linalg.norm(d)), [1, 0, 0], atol=1e-15)


def test_rotation_from_direction_degenerate_and_invalid():
    assert np.array_equal(S.sph_rotation_from_direction([3, 0, 0])[1], np.eye(3))
    assert np.array_equal(S.sph_rotation_from_direction([-1, 0, 0])[1], np.diag([-1.0, -1.0, 1.0]))
    assert S.sph_rotation_from_direction([0, 0, 0])[0] == S.SPH_ERR_ARG
    assert S.sph_rotation_from_direction([np.nan, 0, 1])[0] == S.SPH_ERR_ARG


@pytest.mark.parametrize("seed", range(5))
def test_axis_angle_is_the_printed_rodrigues(seed):
    rng = np.random.default_rng(seed)
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    th = rng.uniform(0, math.pi)
    st, r = S.sph_rotation_axis_angle(n, th)
    assert st == 0
    np.testing.assert_allclose(r, oracle.rodrigues(n, th), atol=1e-15)


def test_check_rotation():
    assert S.sph_check_rotation(3, np.eye(3)) == 0
    assert S.sph_check_rotation(3, np.diag([1.0, 1.0, -1.0])) == S.SPH_ERR_ROTATION   # reflection
    assert S.sph_check_rotation(3, np.eye(3) * 1.01) == S.SPH_ERR_ROTATION
    q = oracle.rotation_2d(0.3)
    assert S.sph_check_rotation(2, q) == 0
    bad = q.copy()
    bad[0, 0] += 1e-6
    assert S.sph_check_rotation(2, bad) == S.SPH_ERR_ROTATION
    assert S.sph_check_rotation(4, q) == S.SPH_ERR_ARG


def _cover_cells(dim, lo, cs, dims, b):
    st, f, ln = S.sph_grid_cover(dim, lo, cs, dims, b.origin, b.rot, b.half, b.margin)
    assert st == 0
    cells = set()
    for a, l in zip(f, ln):
        cells.update(range(int(a), int(a) + int(l)))
    return cells


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("seed", range(4))
def test_grid_cover_holds_every_point_of_the_check_region(dim, seed):
    """Dense random points inside the check region (and on its faces) must bin,
    with the FP32 cell key, into a covered cell -- also when the region sticks
    out of the grid and particles are binned into edge cells."""
    rng = np.random.default_rng(seed)
    dp = 0.01
    cs = 2.6 * dp
    half = np.array([2 * dp, rng.uniform(0.05, 0.2), rng.uniform(0.05, 0.2)])
    margin = cs
    if dim == 2:
        q = oracle.rotation_2d(rng.uniform(-math.pi, math.pi))
    else:
        v = rng.standard_normal(3)
        q = oracle.rotation_from_direction(v)
    origin = rng.uniform(-0.1, 0.1, 3)
    if dim == 2:
        origin[2] = 0
    b = oracle.Buffer(2, tuple(origin), q, tuple(half), margin)
    lo = np.array([-0.25, -0.25, -0.25]) + rng.uniform(-0.01, 0.01, 3)   # region may poke out
    dims = [int(math.ceil(0.5 / cs))] * 3
    cells = _cover_cells(dim, lo, cs, dims, b)
    n = 200000
    L = rng.uniform(-1, 1, size=(n, 3)) * (half + margin)
    face = rng.integers(0, dim, n)        # push a third of them onto a face
    on = rng.uniform(size=n) < 0.33
    L[on, face[on]] = np.sign(L[on, face[on]]) * (half + margin)[face[on]] * (1 - 1e-9)
    if dim == 2:
        L[:, 2] = 0
    P = (L @ q + origin).astype(np.float32)
    lc = oracle.local_coords(dim, b, P[:, 0], P[:, 1], P[:, 2] if dim == 3 else None)
    inside = np.all(np.abs(lc[:, :dim]) < (half + margin)[:dim], axis=1)
    lo32 = np.float32(lo[:dim])
    start, idx = oracle.cell_list(dim, lo32, np.float32(1.0 / cs), dims[:dim], P[:, 0], P[:, 1],
                                  P[:, 2] if dim == 3 else None)
    cell_of = np.empty(n, np.int64)
    cell_of[idx] = np.repeat(np.arange(len(start) - 1), np.diff(start))
    missing = [int(c) for c in cell_of[inside] if int(c) not in cells]
    assert not missing, f"{len(missing)} points of the check region fall in uncovered cells"


def test_grid_cover_is_tight_for_axis_aligned_box():
    # axis-aligned check box [0.1, 0.3] x [0.1, 0.3] on a unit grid of 0.1 cells:
    # only the cells it touches (plus the 1e-2-cell dilation) are listed
    q = np.eye(3)
    st, f, ln = S.sph_grid_cover(2, (0, 0, 0), 0.1, (10, 10, 1), (0.2, 0.2, 0), q, (0.05, 0.05, 0), 0.05)
    assert st == 0
    cells = sorted(c for a, l in zip(f, ln) for c in range(a, a + l))
    assert cells == [ix + 10 * iy for iy in range(0, 4) for ix in range(0, 4)]


def test_guard_band_is_1e4_dp_for_the_pipe():
    dp = 0.001
    g = S.sph_guard_band(3, (0, 0, 1.0), (2 * dp, 0.05 / math.cos(math.radians(35)) + 2 * dp,
                                          0.05 / math.cos(math.radians(35)) + 2 * dp), 2.6 * dp, 2.6 * dp, dp)
    assert g == pytest.approx(1e-4 * dp)


def _fp32_cells(dim, lo, cs, dims, P):
    """Cell coordinates exactly as the kernels bin an FP32 position:
    floor(fl32(fl32(x - fl32(lo)) * fl32(1/cs))), clamped to the grid."""
    lo32 = np.asarray(lo[:dim], dtype=np.float32)
    ic = np.float32(1.0 / cs)
    t = ((P[:, :dim] - lo32).astype(np.float32) * ic).astype(np.float32)
    c = np.floor(t).astype(np.int64)
    return np.clip(c, 0, np.asarray(dims[:dim]) - 1)


WIDE_DP = 0.001
WIDE_CS = 2.6 * WIDE_DP
# 150,000 cells along x, origin 10^6 cells from 0: lo_x rounds to FP32 with an
# error of 0.045 cells, which shifts every binned particle by that much
WIDE_LO = np.array([1e6 * WIDE_CS + 0.37 * WIDE_DP, -8 * WIDE_CS + 0.11 * WIDE_DP, 0.0])
WIDE_DIMS = [150_000, 16, 1]


def misbinned_column(lo, cs, dims, k_start):
    """An FP32 x value that lies 0.012 .. 0.044 cells right of a cell face (in
    exact arithmetic) but is binned into the cell left of that face, near cell
    k_start: (x, cell index of the face)."""
    for k in range(k_start, k_start - 200, -1):
        face = lo[0] + k * cs
        x = np.float32(face)
        while float(x) < face + 0.05 * cs:
            if float(x) > face + 0.012 * cs:
                c = _fp32_cells(2, lo, cs, dims, np.array([[x, 0.0, 0.0]], np.float32))[0, 0]
                if c == k - 1:
                    return float(x), k
            x = np.nextafter(x, np.float32(np.inf))
    raise AssertionError("no misbinned FP32 column")


def test_grid_cover_holds_fp32_binning_on_a_wide_far_grid():
    """A 2-D grid of 150,000 cells along x whose origin lies 10^6 cells from 0: the
    FP32 cell coordinate is off by up to ~0.07 cells there.  (1) An axis-aligned
    outlet whose check region starts just left of an FP32 column that is binned a
    cell too low: those points must bin into a covered cell (a dilation of 1e-2
    cell would miss them).  (2) Random points of an oblique outlet's check region,
    most within a fraction of a cell of its boundary."""
    dp, cs, lo, dims = WIDE_DP, WIDE_CS, WIDE_LO, WIDE_DIMS
    half = np.array([2 * dp, 0.012, 0.0])
    margin = cs
    ext = (half + margin)[:2]
    # (1) adversarial axis-aligned region
    xc, k = misbinned_column(lo, cs, dims, dims[0] - 30)
    origin = np.array([xc - 1e-9 + ext[0], 0.0012, 0.0])
    b = oracle.Buffer(2, tuple(origin), np.eye(3), tuple(half), margin)
    cells = _cover_cells(2, lo, cs, dims, b)
    ys = np.linspace(origin[1] - 0.9 * ext[1], origin[1] + 0.9 * ext[1], 101)
    P = np.zeros((len(ys), 3), np.float32)
    P[:, 0] = np.float32(xc)
    P[:, 1] = ys
    lc = oracle.local_coords(2, b, P[:, 0], P[:, 1], None)
    assert np.all(np.abs(lc[:, :2]) < ext)             # all in the check region
    c = _fp32_cells(2, lo, cs, dims, P)
    assert np.all(c[:, 0] == k - 1)                    # binned left of the region's first cell
    missing = [int(q) for q in c[:, 0] + dims[0] * c[:, 1] if int(q) not in cells]
    assert not missing, f"{len(missing)} points of the check region fall in uncovered cells"
    # (2) oblique region, random points mostly near its boundary
    rng = np.random.default_rng(5)
    q = oracle.rotation_2d(math.radians(-35.0))
    origin = np.array([lo[0] + (dims[0] - 20) * cs, 0.0012, 0.0])
    b = oracle.Buffer(2, tuple(origin), q, tuple(half), margin)
    cells = _cover_cells(2, lo, cs, dims, b)
    n = 400_000
    L = rng.uniform(-1, 1, size=(n, 2)) * ext
    shell = rng.uniform(size=n) < 0.7
    side = rng.integers(0, 2, n)
    depth = rng.uniform(0.0, 0.3 * cs, n)
    L[shell, side[shell]] = np.sign(L[shell, side[shell]]) * (ext[side[shell]] - depth[shell])
    P = np.zeros((n, 3))
    P[:, :2] = L @ q[:2, :2] + origin[:2]
    P = P.astype(np.float32)
    lc = oracle.local_coords(2, b, P[:, 0], P[:, 1], None)
    inside = np.all(np.abs(lc[:, :2]) < ext, axis=1)
    c = _fp32_cells(2, lo, cs, dims, P)
    exact = np.floor((P[:, :2].astype(np.float64) - lo[:2]) / cs).astype(np.int64)
    assert np.count_nonzero(np.any(c != exact, axis=1) & inside) > 1000
    key = c[:, 0] + dims[0] * c[:, 1]
    missing = [int(q) for q in key[inside] if int(q) not in cells]
    assert not missing, f"{len(missing)} points of the check region fall in uncovered cells"


def test_grid_cover_refuses_grids_too_wide_for_fp32_binning():
    # 2^23 cells along x: the relative FP32 error alone reaches 1.5 cells
    dims = [1 << 23, 4, 1]
    st, f, ln = S.sph_grid_cover(2, (0, 0, 0), 1e-3, dims, (0.5, 0.002, 0), np.eye(3), (1e-3, 1e-3, 0), 1e-3)
    assert st == S.SPH_ERR_ARG
