"""Property tests of the oracle on generated inputs (hypothesis): for random
buffer kinds, extents, margins, frames and particle sets placed away from every
threshold, the update in a rotated and translated frame gives the events of the
axis-aligned one (the one-axis test of Section 3 does not depend on the frame),
and the counts balance (N' = N - |D| + |G|, ids stay unique)."""
import math

import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from tests._support import make_state

I3 = np.eye(3)


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(dim=st.sampled_from([2, 3]), kind=st.sampled_from([oracle.INLET, oracle.OUTLET, oracle.BIDIR]),
       seed=st.integers(0, 2 ** 31 - 1), ha=st.floats(0.002, 0.02), hb=st.floats(0.01, 0.1),
       hc=st.floats(0.01, 0.1), mfrac=st.floats(0.3, 2.0), n=st.integers(1, 600))
def test_events_do_not_depend_on_the_frame(dim, kind, seed, ha, hb, hc, mfrac, n):
    rng = np.random.default_rng(seed)
    half = np.array([ha, hb, hc])
    margin = mfrac * ha
    lim = half + 2 * margin
    L = rng.uniform(-lim, lim, size=(n, 3))
    if dim == 2:
        L[:, 2] = 0.0
    ok = np.ones(n, bool)
    for c in range(dim):
        for t in (half[c], half[c] + margin):
            ok &= np.abs(np.abs(L[:, c]) - t) > 1e-4 * ha
    L = L[ok]
    n = L.shape[0]
    if n == 0:
        return
    in_check = np.all(np.abs(L[:, :dim]) < (half + margin)[:dim], axis=1)
    labels = ((rng.uniform(size=n) < 0.5) & in_check).astype(np.int32)
    if dim == 2:
        q = oracle.rotation_2d(rng.uniform(-math.pi, math.pi))
    else:
        d = rng.standard_normal(3)
        q = oracle.rotation_from_direction(d / np.linalg.norm(d))
    origin = rng.uniform(-1.0, 1.0, 3)
    if dim == 2:
        origin[2] = 0.0
    G = L @ q + origin  # r = Q^T r' + O'
    ref = oracle.Buffer(kind, (0, 0, 0), I3, tuple(half), margin)
    rot = oracle.Buffer(kind, tuple(origin), q, tuple(half), margin)
    s_ref = make_state(dim, L[:, :dim], capacity=2 * n + 4, labels=labels)
    s_rot = make_state(dim, G[:, :dim], capacity=2 * n + 4, labels=labels)
    r1 = oracle.update([ref], s_ref)
    r2 = oracle.update([rot], s_rot)
    assert r1.status == r2.status == oracle.OK
    np.testing.assert_array_equal(r1.gen, r2.gen)
    np.testing.assert_array_equal(r1.dele, r2.dele)
    np.testing.assert_array_equal(s_ref.label[: s_ref.n], s_rot.label[: s_rot.n])
    for s, r in ((s_ref, r1), (s_rot, r2)):
        assert s.n == n - len(r.dele) + len(r.gen)
        ids = s.id[: s.n]
        assert len(np.unique(ids)) == s.n
