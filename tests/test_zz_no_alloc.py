"""sph_celllist_build_noalloc (the cell-list build for callers that cannot
allocate: all scratch in a fixed library-owned device array) against the
context's sph_celllist_build on the same positions: cell starts equal, each
cell's set of indices equal (the order inside a cell is free).  Two calls in a
row, the second with fewer particles on a smaller grid; sizes past the maxima
are refused."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests._gpu import make_domain_raw
from tests._support import make_state

pytestmark = pytest.mark.gpu


def _reference(dim, lo, hi, cs, pts):
    """Cell list of the context build (the existing entry point)."""
    from tests.test_parity_gpu import _cell_list
    st = make_state(dim, pts, capacity=len(pts) + 8)
    d = make_domain_raw(dim, lo, hi, cs, 0.01, [], st)
    d.build()
    cs_, ci, dims = _cell_list(d, len(pts))
    d.close()
    return cs_, ci, dims


def _noalloc(dim, lo, cs, dims, pts, capacity):
    import torch
    from paper_2406_16786_amd import sphbuf as S
    dev = torch.device("cuda:0")
    n = len(pts)
    pos = [torch.zeros(capacity, dtype=torch.float32, device=dev) for _ in range(3)]
    for c in range(dim):
        pos[c][:n] = torch.from_numpy(np.ascontiguousarray(pts[:, c], dtype=np.float32)).to(dev)
    n_dev = torch.tensor([n], dtype=torch.int64, device=dev)
    cells = int(np.prod(dims[:dim]))
    start = torch.full((cells + 1,), -7, dtype=torch.int32, device=dev)
    idx = torch.full((capacity,), -7, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    rc = S.sph_celllist_build_noalloc(dim, lo, cs, dims, pos[0].data_ptr(), pos[1].data_ptr(),
                                      pos[2].data_ptr() if dim == 3 else 0, n_dev.data_ptr(), capacity,
                                      start.data_ptr(), idx.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    return rc, start.cpu().numpy(), idx.cpu().numpy()


def _same_cell_lists(ref_s, ref_i, got_s, got_i, n):
    np.testing.assert_array_equal(got_s, ref_s)
    cell_of = np.repeat(np.arange(len(ref_s) - 1), np.diff(ref_s))
    np.testing.assert_array_equal(got_i[:n][np.lexsort((got_i[:n], cell_of))], ref_i[np.lexsort((ref_i, cell_of))])


def test_noalloc_build_matches_the_context_build_twice():
    rng = np.random.default_rng(17)
    # first call: 3-D, 600 k particles (lattice-like plus a crowded cell)
    n1 = 600_000
    pts1 = np.concatenate([rng.uniform((0, 0, 0), (1.0, 0.5, 0.4), (n1 - 3000, 3)),
                           0.5 + rng.uniform(-0.004, 0.004, (3000, 3))])
    lo1, hi1, cs1 = (0.0, 0.0, 0.0), (1.0, 0.5, 0.5), 0.013
    ref_s, ref_i, dims1 = _reference(3, lo1, hi1, cs1, pts1)
    assert int(np.prod(dims1)) <= (1 << 20)
    rc, got_s, got_i = _noalloc(3, lo1, cs1, dims1, pts1, n1 + 100)
    assert rc == 0
    _same_cell_lists(ref_s, ref_i, got_s, got_i, n1)
    # second call: 2-D, fewer particles, a smaller grid
    n2 = 70_000
    pts2 = rng.uniform((-0.3, 0.2), (0.4, 0.6), (n2, 2))
    lo2, hi2, cs2 = (-0.3, 0.2, 0.0), (0.4, 0.6, 0.0), 0.004
    ref_s, ref_i, dims2 = _reference(2, lo2, hi2, cs2, pts2)
    rc, got_s, got_i = _noalloc(2, lo2, cs2, dims2, pts2, n2)
    assert rc == 0
    _same_cell_lists(ref_s, ref_i, got_s, got_i, n2)


def test_noalloc_build_refuses_sizes_past_its_maxima():
    import torch
    from paper_2406_16786_amd import sphbuf as S
    dev = torch.device("cuda:0")
    x = torch.zeros(16, dtype=torch.float32, device=dev)
    n_dev = torch.zeros(1, dtype=torch.int64, device=dev)
    out = torch.zeros(16, dtype=torch.int32, device=dev)
    p = x.data_ptr()
    big = S.SPH_NOALLOC_MAX_PARTICLES + 1
    assert S.sph_celllist_build_noalloc(2, (0, 0, 0), 0.1, (4, 4, 1), p, p, 0, n_dev.data_ptr(), big,
                                        out.data_ptr(), out.data_ptr()) == S.SPH_ERR_ARG
    assert S.sph_celllist_build_noalloc(3, (0, 0, 0), 0.1, (128, 128, 65), p, p, p, n_dev.data_ptr(), 16,
                                        out.data_ptr(), out.data_ptr()) == S.SPH_ERR_ARG
    assert S.sph_celllist_build_noalloc(2, (0, 0, 0), 0.1, (4, 4, 1), p, p, 0, 0, 16,
                                        out.data_ptr(), out.data_ptr()) == S.SPH_ERR_ARG
