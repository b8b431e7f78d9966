"""Error paths of the C ABI on a GPU: every define-time refusal of
sph_buffer_define, the event limit of an update (SPH_ERR_EVENTS, nothing
changed), the refusals of sph_create (bad update path, a grid too wide for FP32
binning), state export / import, and a process that exits with live contexts
and a live batch."""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests._gpu import assert_same_state, make_domain, make_domain_raw, upload_state
from tests._support import make_state, oracle_buffers, oracle_state

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ctx(dim=2, lo=(0, 0, 0), hi=(1, 1, 1), cs=0.05, **kw):
    from paper_2406_16786_amd import sphbuf as S
    st, ctx = S.sph_create(dim, lo, hi, cs, 0.02, 1024, **kw)
    return st, ctx


def test_define_time_errors():
    from paper_2406_16786_amd import sphbuf as S
    st, ctx = _ctx()
    assert st == 0
    q = np.eye(3)
    ok, bid = S.sph_buffer_define(ctx, S.SPH_INLET, (0.1, 0.5, 0), q, (0.04, 0.2, 0), 0.05)
    assert ok == 0 and bid == 1
    # check regions meet: the second box's region reaches into the first's
    assert S.sph_buffer_define(ctx, S.SPH_OUTLET, (0.25, 0.5, 0), q, (0.04, 0.2, 0), 0.05)[0] == S.SPH_ERR_OVERLAP
    # not a rotation: a reflection, a scaled matrix, a NaN
    refl = np.diag([1.0, -1.0, 1.0])
    assert S.sph_buffer_define(ctx, S.SPH_OUTLET, (0.8, 0.5, 0), refl, (0.04, 0.2, 0), 0.05)[0] == \
        S.SPH_ERR_ROTATION
    assert S.sph_buffer_define(ctx, S.SPH_OUTLET, (0.8, 0.5, 0), 1.01 * q, (0.04, 0.2, 0), 0.05)[0] == \
        S.SPH_ERR_ROTATION
    qn = q.copy()
    qn[0, 1] = np.nan
    assert S.sph_buffer_define(ctx, S.SPH_OUTLET, (0.8, 0.5, 0), qn, (0.04, 0.2, 0), 0.05)[0] == S.SPH_ERR_ROTATION
    # bad kind, non-positive or non-finite extents, non-finite origin or margin
    assert S.sph_buffer_define(ctx, 7, (0.8, 0.5, 0), q, (0.04, 0.2, 0), 0.05)[0] == S.SPH_ERR_ARG
    assert S.sph_buffer_define(ctx, S.SPH_OUTLET, (0.8, 0.5, 0), q, (0.0, 0.2, 0), 0.05)[0] == S.SPH_ERR_ARG
    assert S.sph_buffer_define(ctx, S.SPH_OUTLET, (0.8, 0.5, 0), q, (0.04, -0.2, 0), 0.05)[0] == S.SPH_ERR_ARG
    assert S.sph_buffer_define(ctx, S.SPH_OUTLET, (0.8, 0.5, 0), q, (0.04, np.inf, 0), 0.05)[0] == S.SPH_ERR_ARG
    assert S.sph_buffer_define(ctx, S.SPH_OUTLET, (np.nan, 0.5, 0), q, (0.04, 0.2, 0), 0.05)[0] == S.SPH_ERR_ARG
    assert S.sph_buffer_define(ctx, S.SPH_OUTLET, (0.8, 0.5, 0), q, (0.04, 0.2, 0), np.nan)[0] == S.SPH_ERR_ARG
    # none of the refusals took a buffer id
    ok, bid = S.sph_buffer_define(ctx, S.SPH_OUTLET, (0.9, 0.5, 0), q, (0.04, 0.2, 0), 0.05)
    assert ok == 0 and bid == 2
    S.sph_destroy(ctx)


def test_too_many_buffers():
    from paper_2406_16786_amd import sphbuf as S
    st, ctx = _ctx(hi=(4, 1, 1))
    assert st == 0
    for k in range(S.SPH_MAX_BUFFERS):
        ok, bid = S.sph_buffer_define(ctx, S.SPH_OUTLET, (0.1 + 0.25 * k, 0.5, 0), np.eye(3), (0.02, 0.1, 0), 0.02)
        assert ok == 0 and bid == k + 1
    assert S.sph_buffer_define(ctx, S.SPH_OUTLET, (3.9, 0.5, 0), np.eye(3), (0.02, 0.1, 0), 0.02)[0] == \
        S.SPH_ERR_TOO_MANY_BUFFERS
    S.sph_destroy(ctx)


def test_create_refusals():
    from paper_2406_16786_amd import sphbuf as S
    assert _ctx(update_path=5)[0] == S.SPH_ERR_ARG
    assert _ctx(build_method=3)[0] == S.SPH_ERR_ARG
    assert _ctx(build_method=-1)[0] == S.SPH_ERR_ARG
    # 2^23 cells along x: FP32 binning is off by more than a cell there
    st, ctx = S.sph_create(2, (0, 0, 0), ((1 << 23) * 1e-3, 0.004, 0), 1e-3, 4e-4, 1024)
    assert st == S.SPH_ERR_ARG and not ctx
    # the wide far grid of the cover test is accepted (its bound is ~0.07 cells)
    from tests.test_abi_host import WIDE_CS, WIDE_DIMS, WIDE_LO
    hi = WIDE_LO + (np.array(WIDE_DIMS) - 0.5) * WIDE_CS
    st, ctx = S.sph_create(2, WIDE_LO, hi, WIDE_CS, 0.001, 1024)
    assert st == 0
    S.sph_destroy(ctx)


@pytest.mark.parametrize("path", ["merged", "cells", "fullscan"])
def test_event_limit_leaves_state_untouched(path):
    """max_events = 8 and 12 particles beyond the outlet: the update returns
    SPH_ERR_EVENTS and changes nothing; with max_events = 12 it goes through."""
    bufs = [oracle.Buffer(oracle.OUTLET, (0.9, 0.5, 0), np.eye(3), (0.04, 0.3, 0), 0.05)]
    rng = np.random.default_rng(3)
    pts = np.concatenate([rng.uniform((0.1, 0.3), (0.8, 0.7), (200, 2)),
                          np.column_stack([np.full(12, 0.96), np.linspace(0.3, 0.7, 12)])])
    for cap in (8, 12):
        st = make_state(2, pts, capacity=400)
        d = make_domain_raw(2, (0, 0, 0), (1, 1, 0), 0.05, 0.02, bufs, st, max_events=cap,
                            update_path="cells" if path == "cells" else "merged")
        assert d.identify(-1) == 0
        oracle.identify(bufs, st, -1)
        if path == "fullscan":
            gst, g, dl = d.update_fullscan()
        else:
            d.build()
            gst, g, dl = d.update()
        if cap == 8:
            assert gst == 8  # SPH_ERR_EVENTS (the oracle has no event limit)
            assert_same_state(d, st, "refused update")
        else:
            res = oracle.update(bufs, st)
            assert gst == res.status == 0 and dl == 12
            assert_same_state(d, st, "update at the limit")
        d.close()


def test_state_export_import_round_trip():
    from paper_2406_16786_amd import sphbuf as S
    wl = W.channel2d()
    bufs = oracle_buffers(wl)
    st = oracle_state(wl)
    d = make_domain(wl, bufs, st)
    assert oracle.identify(bufs, st, -1)[0] == 0 and d.identify(-1) == 0
    for step in range(5):
        W.advect_host(wl, st.pos, st.n, step)
        upload_state(d, st)
        d.build()
        res = oracle.update(bufs, st)   # the host state follows the device's
        assert d.update()[0] == res.status == 0
    rc, blob = S.sph_state_export(d.ctx)
    assert rc == 0 and len(blob) == S.SPH_STATE_BLOB_BYTES
    rc, nid, nl = S.sph_state_get(d.ctx)
    assert nid == st.next_id and list(nl[: len(bufs)]) == list(res.n_labelled)
    d2 = make_domain(wl, bufs, oracle_state(wl))
    assert S.sph_state_import(d2.ctx, blob) == 0
    rc2, nid2, nl2 = S.sph_state_get(d2.ctx)
    assert nid2 == nid and np.array_equal(nl2, nl)
    bad = bytearray(blob)
    bad[0] ^= 1
    assert S.sph_state_import(d2.ctx, bytes(bad)) == S.SPH_ERR_ARG
    assert S.sph_state_import(d2.ctx, blob[:-8]) == S.SPH_ERR_ARG
    d.close()
    d2.close()


def test_exit_with_live_contexts_and_batch():
    """A program that creates domains (both update paths) and a batch, steps them and
    exits without closing anything ends with status 0."""
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import torch, workloads as W\n"
        "from paper_2406_16786_amd import sphbuf as S\n"
        "from paper_2406_16786_amd.domain import Domain\n"
        "doms = []\n"
        "for i, wl in enumerate(W.hub_batch(3, 2e3, 1e4, seed=9)):\n"
        "    d = Domain(wl.dim, wl.lo, wl.hi, wl.cell_size, wl.dp, wl.capacity, wl.pos, wl.carried, wl.label,\n"
        "               wl.id, wl.n, wl.n, update_path='merged' if i %% 2 else 'cells')\n"
        "    for b in wl.buffers:\n"
        "        q = S.sph_rotation_2d(b.angle)[1] if wl.dim == 2 else S.sph_rotation_from_direction(b.direction)[1]\n"
        "        d.define(b.kind, b.origin, q, b.half, b.margin)\n"
        "    d.identify(-1); d.build(); d.update_async()\n"
        "    doms.append(d)\n"
        "stream = torch.cuda.Stream()\n"
        "torch.cuda.synchronize()\n"
        "st, b = S.sph_batch_create([d.ctx for d in doms], [d.p for d in doms], stream.cuda_stream)\n"
        "assert st == 0 and S.sph_batch_step(b) == 0\n"
        "print('stepped', flush=True)\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    assert "stepped" in r.stdout


def test_exit_after_an_error_with_live_handles():
    """A program that raises with a domain and a batch alive: the exit hook destroys
    them, and the domain's own close() when it is collected afterwards does nothing
    (no second free): the process ends with the error's status 1, not a crash."""
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import torch, workloads as W\n"
        "from paper_2406_16786_amd import sphbuf as S\n"
        "from paper_2406_16786_amd.domain import Domain\n"
        "def run():\n"
        "    wl = W.channel2d()\n"
        "    d = Domain(wl.dim, wl.lo, wl.hi, wl.cell_size, wl.dp, wl.capacity, wl.pos, wl.carried, wl.label,\n"
        "               wl.id, wl.n, wl.n)\n"
        "    for b in wl.buffers:\n"
        "        d.define(b.kind, b.origin, S.sph_rotation_2d(b.angle)[1], b.half, b.margin)\n"
        "    d.identify(-1); d.build(); d.update_async()\n"
        "    stream = torch.cuda.Stream()\n"
        "    torch.cuda.synchronize()\n"
        "    st, b = S.sph_batch_create([d.ctx], [d.p], stream.cuda_stream)\n"
        "    assert st == 0 and S.sph_batch_step(b) == 0\n"
        "    print('stepped', flush=True)\n"
        "    raise RuntimeError('planned')\n"
        "run()\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 1, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    assert "stepped" in r.stdout and "planned" in r.stderr
    assert "double free" not in r.stderr and "corruption" not in r.stderr
