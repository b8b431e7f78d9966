"""Pins of the oracle's boundary conditions (Section 4) and buffer rotation
(Section 5.3) against closed forms, exact special cases and invariants.

Velocity BC: Eqs. 2D/3D_velocity_profile and 2D/3D_velocity_transformation.
Pressure BC: Eq. velocity_correction with Eqs. 2D/3D_normal_transformation, and
Eq. postulate-density for the recycled particles.
Rotating buffer: the rotation step of the sprinkler (Section 5.3).
"""
import math

import numpy as np

import oracle
from tests._support import make_state

I3 = np.eye(3)
# exact quarter turn: X' = y, Y' = -x (Eq. 2D_transformation at theta = 90 degrees)
Q90 = np.array([[0.0, 1.0, 0.0], [-1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
# exact anticlockwise quarter turn of a body about the z axis
M90 = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])

VEL2 = oracle.Fields(vel=(0, 1), rho=2)


def _state2(pts, labels, vel=None, rho=None):
    st = make_state(2, pts, labels=labels, carried=3)
    n = st.n
    if vel is not None:
        st.carried[0][:n] = np.asarray(vel, np.float32)[:, 0]
        st.carried[1][:n] = np.asarray(vel, np.float32)[:, 1]
    if rho is not None:
        st.carried[2][:n] = np.float32(rho)
    return st


# ------------------------------------------------------------ velocity BC ---

def test_parabolic_profile_axis_aligned_closed_form():
    buf = oracle.Buffer(oracle.INLET, (0.0, 0.0), I3, (0.5, 0.5), 0.1)
    bc = oracle.BC(oracle.BC_VELOCITY, oracle.PROFILE_PARABOLIC_Y, u=2.0, radius=0.5)
    st = _state2([(0.1, 0.25), (-0.2, 0.0), (0.3, -0.5), (0.0, 0.0)], [1, 1, 1, 0], vel=[(9, 9)] * 4)
    assert oracle.apply_bc([buf], [bc], VEL2, st) == oracle.OK
    # f = 1 - (Y'/R)^2: 0.75 at Y' = R/2, 1 on the axis, 0 at the wall
    np.testing.assert_array_equal(st.carried[0][:4], np.float32([1.5, 2.0, 0.0, 9.0]))
    np.testing.assert_array_equal(st.carried[1][:4], np.float32([0.0, 0.0, 0.0, 9.0]))


def test_profile_is_mapped_to_global_by_the_transposed_frame():
    # theta = 90 degrees: X' = y, so the inflow points along +y (Eq. 2D_velocity_transformation)
    buf = oracle.Buffer(oracle.INLET, (0.0, 0.0), Q90, (0.5, 0.5), 0.1)
    bc = oracle.BC(oracle.BC_VELOCITY, oracle.PROFILE_PARABOLIC_Y, u=2.0, radius=0.5)
    st = _state2([(-0.25, 0.1)], [1], vel=[(0, 0)])   # X' = 0.1, Y' = 0.25
    assert oracle.apply_bc([buf], [bc], VEL2, st) == oracle.OK
    assert (st.carried[0][0], st.carried[1][0]) == (np.float32(0.0), np.float32(1.5))


def test_plug_profile_points_along_the_buffer_axis_at_any_angle():
    rng = np.random.default_rng(3)
    for theta in rng.uniform(-math.pi, math.pi, 8):
        q = oracle.rotation_2d(theta)
        buf = oracle.Buffer(oracle.INLET, (1.0, 2.0), q, (0.2, 0.4), 0.1)
        bc = oracle.BC(oracle.BC_VELOCITY, oracle.PROFILE_PLUG, u=3.0)
        st = _state2([(1.0, 2.0)], [1], vel=[(0, 0)])
        assert oracle.apply_bc([buf], [bc], VEL2, st) == oracle.OK
        v = np.array([st.carried[0][0], st.carried[1][0]], np.float64)
        np.testing.assert_allclose(v, 3.0 * np.array([math.cos(theta), math.sin(theta)]), atol=1e-6)


def test_pipe_profile_depends_on_the_radius_in_the_cross_section():
    q = oracle.rotation_from_direction((0.0, 0.0, 1.0))     # X' along +z
    buf = oracle.Buffer(oracle.INLET, (0.0, 0.0, 0.0), q, (0.1, 1.0, 1.0), 0.1)
    bc = oracle.BC(oracle.BC_VELOCITY, oracle.PROFILE_PARABOLIC_R, u=1.0, radius=1.0)
    rng = np.random.default_rng(5)
    pts = np.column_stack([rng.uniform(-0.7, 0.7, 50), rng.uniform(-0.7, 0.7, 50), rng.uniform(-0.05, 0.05, 50)])
    st = make_state(3, pts, labels=[1] * 50, carried=3)
    assert oracle.apply_bc([buf], [bc], oracle.Fields(vel=(0, 1, 2)), st) == oracle.OK
    lc = oracle.local_coords(3, buf, st.pos[0][:50], st.pos[1][:50], st.pos[2][:50])
    f = 1.0 - (lc[:, 1] ** 2 + lc[:, 2] ** 2)
    v = np.stack([st.carried[c][:50] for c in range(3)], 1).astype(np.float64)
    np.testing.assert_allclose(v[:, 2], f, rtol=1e-6, atol=1e-7)      # along the axis
    np.testing.assert_allclose(v[:, :2], 0.0, atol=1e-7)             # nothing across it
    # the radius, not Y' alone: same Y', different Z' (X' = z, Y' = y, Z' = -x here)
    st2 = make_state(3, [(0.0, 0.5, 0.0), (-0.5, 0.5, 0.0)], labels=[1, 1], carried=3)
    assert oracle.apply_bc([buf], [bc], oracle.Fields(vel=(0, 1, 2)), st2) == oracle.OK
    np.testing.assert_array_equal(st2.carried[2][:2], np.float32([0.75, 0.5]))


def test_fluid_and_unconstrained_buffers_are_left_alone():
    b1 = oracle.Buffer(oracle.INLET, (0.0, 0.0), I3, (0.5, 0.5), 0.1)
    b2 = oracle.Buffer(oracle.OUTLET, (5.0, 0.0), I3, (0.5, 0.5), 0.1)
    bcs = [oracle.BC(oracle.BC_VELOCITY, oracle.PROFILE_PLUG, u=1.0), oracle.BC()]
    st = _state2([(0.0, 0.0), (0.1, 0.1), (5.0, 0.0), (2.0, 0.0)], [1, 0, 2, 0], vel=[(7, 7)] * 4)
    assert oracle.apply_bc([b1, b2], bcs, VEL2, st) == oracle.OK
    np.testing.assert_array_equal(st.carried[0][:4], np.float32([1.0, 7.0, 7.0, 7.0]))


def test_buffer_particle_outside_its_check_region_is_reported_and_kept():
    buf = oracle.Buffer(oracle.INLET, (0.0, 0.0), I3, (0.5, 0.5), 0.1)
    bc = oracle.BC(oracle.BC_VELOCITY, oracle.PROFILE_PLUG, u=1.0)
    st = _state2([(0.0, 0.0), (3.0, 0.0)], [1, 1], vel=[(7, 7)] * 2)
    assert oracle.apply_bc([buf], [bc], VEL2, st) == oracle.ERR_CFL
    np.testing.assert_array_equal(st.carried[0][:2], np.float32([1.0, 7.0]))


# ------------------------------------------------------------ pressure BC ---

def test_projection_on_the_normal_closed_forms():
    bc = oracle.BC(oracle.BC_PRESSURE, p_b=0.0, rho0=1.0, c0=1.0)
    st = _state2([(0.0, 0.0)], [1], vel=[(3.0, 1.0)])
    assert oracle.apply_bc([oracle.Buffer(oracle.OUTLET, (0, 0), I3, (0.5, 0.5), 0.1)], [bc], VEL2, st) == 0
    assert (st.carried[0][0], st.carried[1][0]) == (np.float32(3.0), np.float32(0.0))
    st = _state2([(0.0, 0.0)], [1], vel=[(3.0, 1.0)])
    assert oracle.apply_bc([oracle.Buffer(oracle.OUTLET, (0, 0), Q90, (0.5, 0.5), 0.1)], [bc], VEL2, st) == 0
    assert (st.carried[0][0], st.carried[1][0]) == (np.float32(0.0), np.float32(1.0))


def test_projection_invariants_at_arbitrary_angles():
    rng = np.random.default_rng(9)
    bc = oracle.BC(oracle.BC_PRESSURE, p_b=0.0, rho0=1.0, c0=1.0)
    for theta in rng.uniform(-math.pi, math.pi, 10):
        q = oracle.rotation_2d(theta)
        buf = oracle.Buffer(oracle.OUTLET, (0.0, 0.0), q, (0.5, 0.5), 0.1)
        v0 = rng.normal(size=2)
        st = _state2([(0.0, 0.0)], [1], vel=[v0])
        assert oracle.apply_bc([buf], [bc], VEL2, st) == 0
        v = np.array([st.carried[0][0], st.carried[1][0]], np.float64)
        uh = np.array([math.cos(theta), math.sin(theta)])
        assert abs(v[0] * uh[1] - v[1] * uh[0]) < 1e-6 * (1 + np.abs(v0).max())     # parallel to u_hat
        assert abs(v @ uh - np.float32(v0) @ uh) < 1e-6 * (1 + np.abs(v0).max())    # normal part kept
        first = v.copy()
        assert oracle.apply_bc([buf], [bc], VEL2, st) == 0                           # idempotent (FP32)
        np.testing.assert_allclose([st.carried[0][0], st.carried[1][0]], first, rtol=1e-6, atol=1e-7)


def test_recycled_particle_takes_the_boundary_density():
    """Eq. postulate-density: rho = rho0 + p_b / c0^2 for the recycled particle of a
    pressure inlet; its duplicate keeps the old state, and a velocity inlet keeps
    the density (Section 4.2)."""
    for kind, expect in ((oracle.BC_PRESSURE, np.float32(1000.5)), (oracle.BC_VELOCITY, np.float32(999.0))):
        buf = oracle.Buffer(oracle.INLET, (0.5, 0.5), I3, (0.5, 0.5), 0.25)
        bc = oracle.BC(kind, oracle.PROFILE_PLUG, u=1.0, p_b=50.0, rho0=1000.0, c0=10.0)
        st = _state2([(1.125, 0.5), (0.25, 0.5)], [1, 1], vel=[(1, 0)] * 2, rho=999.0)
        res = oracle.update([buf], st, [bc], VEL2)
        assert res.status == 0 and list(res.gen) == [0]
        assert st.n == 3
        assert st.carried[2][0] == expect            # the recycled original
        assert st.carried[2][2] == np.float32(999.0)  # its duplicate
        assert st.carried[2][1] == np.float32(999.0)  # not recycled
        assert st.pos[0][0] == np.float32(0.125)


# --------------------------------------------------------------- rotation ---

def test_quarter_turn_about_a_centre_closed_form():
    bufs = [oracle.Buffer(oracle.INLET, (2.0, 1.0, 0.0), I3, (0.25, 0.25, 0.0), 0.125)]
    st = _state2([(2.0, 1.0), (2.125, 1.0625), (5.0, 5.0)], [1, 1, 0], vel=[(1, 0), (0.5, 0.25), (7, 7)])
    assert oracle.rotate_buffer(bufs, 1, (1.0, 1.0), M90, VEL2, st) == oracle.OK
    np.testing.assert_array_equal(np.stack([st.pos[0][:3], st.pos[1][:3]], 1),
                                  np.float32([[1.0, 2.0], [0.9375, 2.125], [5.0, 5.0]]))
    np.testing.assert_array_equal(np.stack([st.carried[0][:3], st.carried[1][:3]], 1),
                                  np.float32([[0.0, 1.0], [-0.25, 0.5], [7.0, 7.0]]))
    np.testing.assert_array_equal(np.asarray(bufs[0].origin)[:2], [1.0, 2.0])
    np.testing.assert_array_equal(bufs[0].rot, Q90)          # X' now points along +y


def test_four_quarter_turns_are_the_identity():
    bufs = [oracle.Buffer(oracle.INLET, (2.0, 1.0, 0.0), I3, (0.25, 0.25, 0.0), 0.125)]
    pts = [(2.0, 1.0), (2.125, 1.0625), (1.875, 0.8125)]
    st = _state2(pts, [1, 1, 1], vel=[(1, 0), (0.5, 0.25), (-2, 3)])
    before = st.copy()
    for _ in range(4):
        assert oracle.rotate_buffer(bufs, 1, (1.0, 1.0), M90, VEL2, st) == oracle.OK
    for c in range(2):
        np.testing.assert_array_equal(st.pos[c][:3], before.pos[c][:3])
        np.testing.assert_array_equal(st.carried[c][:3], before.carried[c][:3])
    np.testing.assert_array_equal(bufs[0].rot, I3)


def test_rotation_keeps_local_coordinates_and_events():
    """A rigid turn moves the frame with the particles: local coordinates are kept
    (to FP32 rounding) and an update after the turn sees the same crossing."""
    rng = np.random.default_rng(2)
    n_hat = rng.normal(size=3)
    n_hat /= np.linalg.norm(n_hat)
    m = oracle.rodrigues(n_hat, 0.7)
    q = oracle.rotation_from_direction((1.0, 0.3, -0.2))
    bufs = [oracle.Buffer(oracle.INLET, (0.5, 0.2, 0.1), q, (0.05, 0.2, 0.2), 0.05)]
    loc = np.column_stack([rng.uniform(-0.049, 0.049, 40), rng.uniform(-0.19, 0.19, 40), rng.uniform(-0.19, 0.19, 40)])
    loc[0, 0] = 0.07                                    # one particle past X' = a/2
    pts = loc @ q + np.array([0.5, 0.2, 0.1])           # r = Q^T r' + O'
    st = make_state(3, pts, labels=[1] * 40, carried=3)
    before = oracle.local_coords(3, bufs[0], *[st.pos[c][:40] for c in range(3)])
    assert oracle.rotate_buffer(bufs, 1, (0.0, 0.0, 0.0), m, oracle.Fields(vel=(0, 1, 2)), st) == oracle.OK
    after = oracle.local_coords(3, bufs[0], *[st.pos[c][:40] for c in range(3)])
    np.testing.assert_allclose(after, before, atol=2e-7)
    res = oracle.update(bufs, st)
    assert res.status == 0 and list(res.gen) == [0]


def test_rotation_reports_buffer_particles_outside_the_check_region():
    bufs = [oracle.Buffer(oracle.INLET, (2.0, 1.0, 0.0), I3, (0.25, 0.25, 0.0), 0.125)]
    st = _state2([(2.0, 1.0), (4.0, 1.0)], [1, 1], vel=[(0, 0)] * 2)
    assert oracle.rotate_buffer(bufs, 1, (1.0, 1.0), M90, VEL2, st) == oracle.ERR_CFL
    assert (st.pos[0][1], st.pos[1][1]) == (np.float32(4.0), np.float32(1.0))
    assert (st.pos[0][0], st.pos[1][0]) == (np.float32(1.0), np.float32(2.0))
