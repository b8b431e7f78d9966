"""GPU parity of the batched path: many independent hub-and-spoke domains (2-D
and 3-D, 1-6 buffers each) stepped together -- five launches per step for all
domains, directly or as a replayed HIP graph -- against the FP64 oracle run
domain by domain; with the domains' contexts created for the cover-cell walk and
for the merged step (the batch runs its own launches either way)."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests._gpu import assert_same_state, make_domain, upload_state
from tests._support import oracle_buffers, oracle_state

pytestmark = pytest.mark.gpu


def _sparse(wl):
    dims = np.ceil((np.array(wl.hi[: wl.dim]) - np.array(wl.lo[: wl.dim])) / wl.cell_size)
    return 3 if wl.dim == 3 and np.prod(dims) > 2 * wl.n else 0


def _setup(wls):
    import torch
    from paper_2406_16786_amd import sphbuf as S
    doms, bufs, states = [], [], []
    for wl in wls:
        b = oracle_buffers(wl)
        st = oracle_state(wl)
        d = make_domain(wl, b, st, brick_log2=_sparse(wl))
        assert oracle.identify(b, st, -1)[0] == 0 and d.identify(-1) == 0
        doms.append(d)
        bufs.append(b)
        states.append(st)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    st, batch = S.sph_batch_create([d.ctx for d in doms], [d.p for d in doms], stream.cuda_stream)
    assert st == 0
    return doms, bufs, states, batch, stream


def _run(wls, steps, mode, tune=False):
    import torch
    from paper_2406_16786_amd import sphbuf as S
    doms, bufs, states, batch, stream = _setup(wls)
    assert S.sph_batch_set_mode(batch, mode) == 0
    if tune:
        st, m, ppb, ms = S.sph_batch_tune(batch, 1, None)
        assert st == 0 and m in (0, 1) and ppb >= 1024
        # tuning ran real updates: bring the oracle to the same point
        torch.cuda.synchronize()
        for d, b, s in zip(doms, bufs, states):
            pos, car, lab, ids, n = d.download()
            for a, c in zip(s.pos + s.carried + [s.label, s.id], pos + car + [lab, ids]):
                a[:] = c
            s.n = n
            s.next_id = int(S.sph_state_get(d.ctx)[1])
    for step in range(steps):
        for wl, s, d in zip(wls, states, doms):
            W.advect_host(wl, s.pos, s.n, step)
            upload_state(d, s)
        torch.cuda.synchronize()
        assert S.sph_batch_step(batch) == 0
        st, res = S.sph_batch_results(batch, len(doms))
        assert st == 0
        for k, (d, b, s) in enumerate(zip(doms, bufs, states)):
            ro = oracle.update(b, s)
            assert res[k].status == ro.status == 0, (step, k, res[k].status, ro.status)
            _, gg, dd = d.events()
            np.testing.assert_array_equal(gg, ro.gen, err_msg=f"step {step} domain {k}")
            np.testing.assert_array_equal(dd, ro.dele, err_msg=f"step {step} domain {k}")
            assert res[k].n_after == s.n
            assert_same_state(d, s, f"step {step} domain {k}")
    S.sph_batch_destroy(batch)
    for d in doms:
        d.close()


@pytest.fixture(params=["cells", "merged"])
def path(request, monkeypatch):
    """The update path of the domains (set when each domain is created)."""
    import tests._gpu as G
    monkeypatch.setattr(G, "UPDATE_PATH", request.param)
    return request.param


@pytest.mark.parametrize("mode", [0, 1])
def test_small_batch_matches_oracle(mode, path):
    _run(W.hub_batch(8, 2e3, 4e4), 12, mode)


def test_batch_after_autotuning(path):
    _run(W.hub_batch(6, 2e3, 2e4, seed=11), 4, 1, tune=True)


def test_full_batch_two_steps(path):
    """64 domains, particle counts log-uniform over 10k-2M (about 27.6 M in all)."""
    _run(W.hub_batch(), 2, 1)


def test_graph_capture_and_launch_calls():
    """sph_batch_graph_capture records the step, sph_batch_graph_launch replays it:
    the same results as stepping in launch mode."""
    import torch
    from paper_2406_16786_amd import sphbuf as S
    wls = W.hub_batch(4, 2e3, 1e4, seed=3)
    doms, bufs, states, batch, stream = _setup(wls)
    assert S.sph_batch_graph_capture(batch) == 0
    for step in range(6):
        for wl, s, d in zip(wls, states, doms):
            W.advect_host(wl, s.pos, s.n, step)
            upload_state(d, s)
        torch.cuda.synchronize()
        assert S.sph_batch_graph_launch(batch) == 0
        st, res = S.sph_batch_results(batch, len(doms))
        assert st == 0
        for k, (d, b, s) in enumerate(zip(doms, bufs, states)):
            ro = oracle.update(b, s)
            assert res[k].status == ro.status == 0
            assert_same_state(d, s, f"step {step} domain {k}")
    S.sph_batch_destroy(batch)
    for d in doms:
        d.close()


@pytest.mark.parametrize("change", ["define", "fields"])
def test_batch_refuses_to_step_after_a_member_changed(change):
    """A batch bakes its members' grid arrays, run-list arrays and field roles into
    its launch tables: after a new buffer or a new density field on a member it
    refuses to step (SPH_ERR_STATE, nothing launched) and the particle arrays stay
    as they were; a new batch steps again."""
    import torch
    from paper_2406_16786_amd import sphbuf as S
    wls = W.hub_batch(3, 2e3, 1e4, seed=7)
    doms, bufs, states, batch, stream = _setup(wls)
    d0 = doms[0]
    if change == "define":
        far = [0.9 * h for h in wls[0].hi]
        assert S.sph_buffer_define(d0.ctx, S.SPH_OUTLET, far, np.eye(3), [1e-3, 1e-3, 1e-3], 1e-3)[0] == 0
    else:
        assert S.sph_set_fields(d0.ctx, [0, 1, 2][: wls[0].dim], 0) == 0
    torch.cuda.synchronize()
    before = [d.download() for d in doms]
    assert S.sph_batch_step(batch) == S.SPH_ERR_STATE
    assert S.sph_batch_graph_launch(batch) == S.SPH_ERR_STATE
    torch.cuda.synchronize()
    for d, b4 in zip(doms, before):
        after = d.download()
        for x, y in zip(b4[0] + b4[1] + [b4[2], b4[3]], after[0] + after[1] + [after[2], after[3]]):
            np.testing.assert_array_equal(x, y)
    S.sph_batch_destroy(batch)
    st, batch2 = S.sph_batch_create([d.ctx for d in doms], [d.p for d in doms], stream.cuda_stream)
    assert st == 0 and S.sph_batch_step(batch2) == 0
    torch.cuda.synchronize()
    S.sph_batch_destroy(batch2)
    for d in doms:
        d.close()


def test_batch_steps_after_a_member_turned():
    """A turn recomputes the member's cover on the device, in the arrays the batch
    already holds: the batch keeps stepping, and every domain matches the oracle
    (with the turned buffer's frame)."""
    import math
    import torch
    from paper_2406_16786_amd import sphbuf as S
    wls = W.hub_batch(3, 2e3, 1e4, seed=7)
    doms, bufs, states, batch, stream = _setup(wls)
    fields = [oracle.Fields(vel=tuple(range(w.dim)), rho=-1) for w in wls]
    for d, w in zip(doms, wls):
        d.set_fields(list(range(w.dim)), -1)
    S.sph_batch_destroy(batch)   # field roles changed: a new batch
    st, batch = S.sph_batch_create([d.ctx for d in doms], [d.p for d in doms], stream.cuda_stream)
    assert st == 0
    for step in range(8):
        for wl, s, d in zip(wls, states, doms):
            W.advect_host(wl, s.pos, s.n, step)
            upload_state(d, s)
        torch.cuda.synchronize()
        assert S.sph_batch_step(batch) == 0
        st, res = S.sph_batch_results(batch, len(doms))
        for k, (d, b, s) in enumerate(zip(doms, bufs, states)):
            ro = oracle.update(b, s)
            assert res[k].status == ro.status == 0, (step, k)
            assert_same_state(d, s, f"step {step} domain {k}")
        # turn the first buffer of domain 0 a little about its own origin
        d0, w0 = doms[0], wls[0]
        m = np.eye(3)
        th = math.radians(0.7)
        m[0, 0], m[0, 1], m[1, 0], m[1, 1] = math.cos(th), -math.sin(th), math.sin(th), math.cos(th)
        c = list(bufs[0][0].origin)[: w0.dim]
        d0.build()
        assert d0.rotate(1, c, m) == oracle.rotate_buffer(bufs[0], 1, c, m, fields[0], states[0]) == 0
        assert_same_state(d0, states[0], f"step {step} turn")
        torch.cuda.synchronize()
    S.sph_batch_destroy(batch)
    for d in doms:
        d.close()
