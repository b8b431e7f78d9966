"""Long runs at full size, as the benchmark runs them: the GPU advances the
particles itself (prescribed velocity, seeded noise) and the FP64 oracle is fed
the GPU's own pre-update state at every checked step (snapshot mode).  The
branching network crosses its first flow reversal (period 200 steps: the flow
turns at step 100), so every bidirectional buffer both generates and deletes;
the pipe is checked late in its run, when the particles have left their
initial lattice order."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests._gpu import advect_device, host_state, make_domain
from tests._support import oracle_buffers, oracle_state

pytestmark = pytest.mark.gpu


def _long_run(wl, steps, check_from, full_every, brick_log2=0):
    import torch
    bufs = oracle_buffers(wl)
    d = make_domain(wl, bufs, oracle_state(wl), brick_log2=brick_log2)
    assert d.identify(-1) == 0
    gen = torch.Generator(device=d.device)
    nd = ng = 0
    gen_at, del_at = set(), set()
    for s in range(steps):
        check = s >= check_from
        full = check and ((s - check_from) % full_every == 0 or s == steps - 1)
        if check:
            ref = host_state(d, None if full else 0)   # positions and labels are what the events depend on
        d.build()
        gst, g, dl = d.update()
        assert gst == 0, (s, gst)
        if check:
            res = oracle.update(bufs, ref)
            assert res.status == 0, (s, res.status)
            _, gg, dd = d.events()
            np.testing.assert_array_equal(gg, res.gen, err_msg=f"step {s} generated")
            np.testing.assert_array_equal(dd, res.dele, err_msg=f"step {s} deleted")
            rs, r = d.result()
            assert r.n_after == ref.n and r.next_id == ref.next_id, s
            assert list(r.n_labelled[: len(bufs)]) == list(res.n_labelled), s
            if full:
                got = host_state(d)
                n = ref.n
                for a, b in zip(got.pos + got.carried + [got.label, got.id],
                                ref.pos + ref.carried + [ref.label, ref.id]):
                    np.testing.assert_array_equal(a[:n], b[:n], err_msg=f"step {s} arrays")
                print(f"step {s}: N = {n}, generated {len(res.gen)}, deleted {len(res.dele)} -- all arrays equal",
                      flush=True)
            ng += len(res.gen)
            nd += len(res.dele)
            if len(res.gen):
                gen_at.add(s)
            if len(res.dele):
                del_at.add(s)
        advect_device(wl, d, s, gen)
    d.close()
    return ng, nd, gen_at, del_at


def test_tree_full_size_across_the_flow_reversal():
    """16.1 M particles, brick-sparse grid, four bidirectional buffers, steps
    0-129: events every step, every array every 25 steps."""
    wl = W.tree3d()
    ng, nd, gen_at, del_at = _long_run(wl, 130, 0, 25, brick_log2=3)
    assert ng > 0 and nd > 0
    # before the reversal the trunk generates and the leaves delete; after it (step
    # > 100) the flow runs backwards: both kinds of event on both sides of it
    assert any(s < 100 for s in gen_at) and any(s > 105 for s in gen_at)
    assert any(s < 100 for s in del_at) and any(s > 105 for s in del_at)


def test_pipe_full_size_late_states():
    """7.86 M particles: 400 steps on the GPU alone, then steps 400-459 checked
    (events every step, every array every 10 steps)."""
    wl = W.pipe3d()
    ng, nd, _, _ = _long_run(wl, 460, 400, 10)
    assert ng > 0 and nd > 0
