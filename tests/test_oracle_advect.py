"""Pins of the oracle's kinematic transport (oracle/advect.py): the velocity
against finite differences of its streamfunction, zero normal velocity on
the box, zero divergence, the midpoint rule's third-order local error against
a tight ODE reference, the clamp, and the loop step with no motion (M2P then
P2M reproduce a linear mesh field)."""
import numpy as np
from scipy.integrate import solve_ivp

from oracle import Mesh
from oracle.advect import kinematic_step, midpoint_step, velocity

MESH = Mesh(12, 8, 1.0 / 8, x0=-0.25, y0=0.5)   # a 1.5 x 1 box off the origin
AMP = 0.3


def _psi(p):
    lx, ly = MESH.nx * MESH.H, MESH.ny * MESH.H
    return AMP * np.sin(np.pi * (p[:, 0] - MESH.x0) / lx) * np.sin(np.pi * (p[:, 1] - MESH.y0) / ly)


def _inside(n, seed=0):
    rng = np.random.default_rng(seed)
    lo = np.array([MESH.x0, MESH.y0])
    return lo + rng.random((n, 2)) * np.array([MESH.nx * MESH.H, MESH.ny * MESH.H])


def test_velocity_is_the_curl_of_the_streamfunction():
    p = _inside(50)
    e = 1e-6
    ex, ey = np.array([e, 0.0]), np.array([0.0, e])
    u_fd = (_psi(p + ey) - _psi(p - ey)) / (2 * e)
    v_fd = -(_psi(p + ex) - _psi(p - ex)) / (2 * e)
    u = velocity(MESH, AMP, p)
    assert np.abs(u[:, 0] - u_fd).max() < 1e-8
    assert np.abs(u[:, 1] - v_fd).max() < 1e-8


def test_no_normal_velocity_on_the_walls_and_no_divergence():
    t = np.linspace(0, 1, 17)
    x1, y1 = MESH.x0 + MESH.nx * MESH.H, MESH.y0 + MESH.ny * MESH.H
    ys = MESH.y0 + t * (y1 - MESH.y0)
    xs = MESH.x0 + t * (x1 - MESH.x0)
    for x in (MESH.x0, x1):
        assert np.abs(velocity(MESH, AMP, np.stack([np.full_like(ys, x), ys], 1))[:, 0]).max() < 1e-15
    for y in (MESH.y0, y1):
        assert np.abs(velocity(MESH, AMP, np.stack([xs, np.full_like(xs, y)], 1))[:, 1]).max() < 1e-15
    p = _inside(40, 1)
    e = 1e-6
    div = ((velocity(MESH, AMP, p + [e, 0])[:, 0] - velocity(MESH, AMP, p - [e, 0])[:, 0])
           + (velocity(MESH, AMP, p + [0, e])[:, 1] - velocity(MESH, AMP, p - [0, e])[:, 1])) / (2 * e)
    assert np.abs(div).max() < 1e-7


def test_midpoint_local_error_is_third_order():
    # points away from the walls, where the clamp would act
    rng = np.random.default_rng(2)
    size = np.array([MESH.nx * MESH.H, MESH.ny * MESH.H])
    p0 = np.array([MESH.x0, MESH.y0]) + size * (0.2 + 0.6 * rng.random((8, 2)))

    def exact(p, dt):
        out = []
        for q in p:
            s = solve_ivp(lambda t, y: velocity(MESH, AMP, y[None])[0], (0, dt), q, method="DOP853",
                          rtol=1e-13, atol=1e-15)
            out.append(s.y[:, -1])
        return np.array(out)

    errs = []
    for dt in (0.08, 0.04, 0.02):
        errs.append(np.abs(midpoint_step(MESH, AMP, dt, p0) - exact(p0, dt)).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 6.5 < r1 < 9.5 and 6.5 < r2 < 9.5, errs


def test_clamp_keeps_particles_in_the_box():
    p = _inside(400, 3)
    q = midpoint_step(MESH, 40.0, 0.5, p)
    x1, y1 = MESH.x0 + MESH.nx * MESH.H, MESH.y0 + MESH.ny * MESH.H
    assert q[:, 0].min() >= MESH.x0 and q[:, 0].max() <= x1
    assert q[:, 1].min() >= MESH.y0 and q[:, 1].max() <= y1


def test_loop_step_without_motion_keeps_a_linear_mesh_field():
    mesh = Mesh(8, 8, 1.0 / 8)
    rng = np.random.default_rng(4)
    g = (np.arange(32) + 0.5) / 32
    X, Y = np.meshgrid(g, g)
    pos = np.stack([X.ravel(), Y.ravel()], 1) + (rng.random((1024, 2)) - 0.5) * 0.3 / 32
    nodes = mesh.nodes()
    field = np.stack([1.0 + 2.0 * nodes[:, 0] - 0.5 * nodes[:, 1], nodes[:, 1]], 1)
    new_pos, new_field = kinematic_step(mesh, 1.0 / 32, 0.0, 0.01, pos, field)
    assert np.array_equal(new_pos, pos)
    assert np.abs(new_field - field).max() < 1e-11


def test_periodic_flow_is_the_curl_of_its_streamfunction_and_periodic():
    from oracle import Mesh
    from oracle.advect import velocity
    m = Mesh(8, 8, 0.25, -1.0, -1.0)
    L = 2.0
    amp = 0.3
    rng = np.random.default_rng(1)
    p = rng.uniform(-1.0, 1.0, size=(50, 2))

    def psi(x, y):
        return amp * np.cos(2 * np.pi * (x + 1.0) / L) * np.cos(2 * np.pi * (y + 1.0) / L)

    e = 1e-6
    u = velocity(m, amp, p, periodic=True)
    fu = (psi(p[:, 0], p[:, 1] + e) - psi(p[:, 0], p[:, 1] - e)) / (2 * e)
    fv = -(psi(p[:, 0] + e, p[:, 1]) - psi(p[:, 0] - e, p[:, 1])) / (2 * e)
    assert np.abs(u[:, 0] - fu).max() < 1e-8 and np.abs(u[:, 1] - fv).max() < 1e-8
    for shift in ((L, 0.0), (0.0, -L), (L, L)):
        assert np.abs(velocity(m, amp, p + shift, periodic=True) - u).max() < 1e-12


def test_periodic_step_is_the_free_step_modulo_the_period():
    """Wrapped positions lie in the box and equal the unclamped midpoint
    step up to whole periods; particles near the sides cross them."""
    from oracle import Mesh
    from oracle.advect import midpoint_step, velocity
    m = Mesh(8, 8, 0.25, -1.0, -1.0)
    L = 2.0
    rng = np.random.default_rng(2)
    p = rng.uniform(-1.0, 1.0, size=(400, 2))
    amp, dt = 0.5, 0.4
    free = p + dt * velocity(m, amp, p + 0.5 * dt * velocity(m, amp, p, True), True)
    got = midpoint_step(m, amp, dt, p, periodic=True)
    assert (got >= -1.0).all() and (got < 1.0).all()
    k = (free - got) / L
    assert np.abs(k - np.rint(k)).max() < 1e-12
    assert np.abs(np.rint(k)).sum() > 0  # some particles crossed a side
