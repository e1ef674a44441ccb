"""Pins for the oracle's M2P (eq. m2p, linear FE on the fixed mesh) and for
the derivatives of P2M and M2P (complex step vs central differences of the
forward construction)."""
import numpy as np
import pytest

import workloads as wl
from oracle import Mesh, P2MOracle, m2p, m2p_matrix, m2p_grad_pos, DomainError
from oracle.adjoint import p2m_grad_pos, roundtrip


def test_m2p_reproduces_linear_fields_exactly():
    rng = np.random.default_rng(0)
    mesh = Mesh(17, 11, 0.0625, -0.3, 0.2)
    pos = np.stack([rng.uniform(-0.3, -0.3 + 17 * 0.0625, 5000),
                    rng.uniform(0.2, 0.2 + 11 * 0.0625, 5000)], 1)
    nodes = mesh.nodes()
    for a, bx, by in [(1.0, 0, 0), (0.3, 2.0, -1.5), (-2.0, 0.25, 4.0)]:
        f = a + bx * nodes[:, 0] + by * nodes[:, 1]
        got = m2p(mesh, f[:, None], pos)[:, 0]
        assert np.abs(got - (a + bx * pos[:, 0] + by * pos[:, 1])).max() < 1e-13


def test_m2p_hand_computed_weights_and_node_values():
    mesh = Mesh(4, 4, 0.25)
    # cell (0,0), xi = 0.25, eta = 0.75 -> upper-left triangle
    # nodes (0,0), (1,1), (0,1) with weights (1-eta, xi, eta-xi) = (0.25, 0.25, 0.5)
    M = m2p_matrix(mesh, np.array([[0.0625, 0.1875]])).toarray()[0]
    want = np.zeros(25)
    want[0], want[6], want[5] = 0.25, 0.25, 0.5
    assert np.array_equal(M, want)
    # cell (2,1), xi = 0.5, eta = 0.25 -> lower-right: (1-xi, xi-eta, eta)
    M = m2p_matrix(mesh, np.array([[0.625, 0.3125]])).toarray()[0]
    want = np.zeros(25)
    want[1 * 5 + 2], want[1 * 5 + 3], want[2 * 5 + 3] = 0.5, 0.25, 0.25
    assert np.array_equal(M, want)
    # particles on nodes (including the top/right boundary) return node values
    nodes = mesh.nodes()
    vals = np.arange(25, dtype=float)[:, None] * 1.5 - 3.0
    assert np.array_equal(m2p(mesh, vals, nodes), vals)


def test_m2p_domain_error():
    mesh = Mesh(4, 4, 0.25)
    with pytest.raises(DomainError):
        m2p(mesh, np.zeros((25, 1)), np.array([[0.5, 1.0000001]]))


def test_m2p_error_order_two_on_taylor_green():
    Hs, errs = [], []
    rng = np.random.default_rng(9)
    pos = rng.uniform(0, 1, (20000, 2))
    for n in (16, 32, 64, 128):
        mesh = Mesh(n, n, 1.0 / n)
        nodes = mesh.nodes()
        got = m2p(mesh, wl.tg_u(nodes[:, 0], nodes[:, 1])[:, None], pos)[:, 0]
        errs.append(np.abs(got - wl.tg_u(pos[:, 0], pos[:, 1])).max())
        Hs.append(1.0 / n)
    slope = np.polyfit(np.log(Hs), np.log(errs), 1)[0]
    assert 1.8 <= slope <= 2.2


def test_m2p_grad_pos_central_differences():
    rng = np.random.default_rng(2)
    mesh = Mesh(8, 8, 0.125)
    nodes = mesh.nodes()
    mv = np.stack([wl.tg_u(nodes[:, 0], nodes[:, 1]), wl.quad_q(nodes[:, 0], nodes[:, 1])], 1)
    pos = rng.uniform(0.01, 0.99, (300, 2))
    g = rng.normal(size=(300, 2))
    ana = m2p_grad_pos(mesh, mv, pos, g)
    d = 1e-7
    for k in range(2):
        e = np.zeros(2)
        e[k] = d
        fp = (m2p(mesh, mv, pos + e) * g).sum(1)
        fm = (m2p(mesh, mv, pos - e) * g).sum(1)
        fd = (fp - fm) / (2 * d)
        # skip particles whose triangle changes within the step
        tx, ty = pos[:, 0] / 0.125, pos[:, 1] / 0.125
        fr = np.minimum(np.abs(tx - np.round(tx)), np.abs(ty - np.round(ty)))
        fr = np.minimum(fr, np.abs((tx - np.floor(tx)) - (ty - np.floor(ty))))
        ok = fr > 1e-5
        assert ok.sum() > 250
        assert np.abs(fd - ana[:, k])[ok].max() < 1e-6


def _structure(orc):
    W, info = orc.matrix()
    return W, (W != 0).astype(np.int8), info["closure"].copy()


@pytest.fixture(scope="module")
def small():
    c = wl.small_cloud(8, 2, 0.25, seed=31, channels=("u", "q"))
    mesh = Mesh.from_spec(c.mesh)
    return c, mesh, P2MOracle(c.pos, mesh, c.h)


def test_p2m_grad_pos_complex_step_vs_central_differences(small):
    c, mesh, orc = small
    rng = np.random.default_rng(8)
    gbar = rng.normal(size=(mesh.n_nodes, 2))
    grad = p2m_grad_pos(orc, c.vals, gbar)
    W0, pat0, cl0 = _structure(orc)
    d = 1e-6
    used = 0
    for mu in rng.choice(c.N, 40, replace=False):
        for k in range(2):
            pp, pm = c.pos.copy(), c.pos.copy()
            pp[mu, k] += d
            pm[mu, k] -= d
            op, om = P2MOracle(pp, mesh, c.h), P2MOracle(pm, mesh, c.h)
            Wp, patp, clp = _structure(op)
            Wm, patm, clm = _structure(om)
            if (patp != pat0).nnz or (patm != pat0).nnz or (clp != cl0).any() or (clm != cl0).any():
                continue   # a Delaunay flip or kNN change inside the step
            fd = (((Wp - Wm) @ c.vals) * gbar).sum() / (2 * d)
            assert abs(fd - grad[mu, k]) <= 1e-6 * max(1.0, abs(grad[mu, k]))
            used += 1
    assert used >= 60


def test_roundtrip_gradients_central_differences(small):
    c, mesh, orc = small
    nodes = mesh.nodes()
    f = np.stack([wl.tg_u(nodes[:, 0] - 0.05, nodes[:, 1] + 0.03),
                  wl.tg_v(nodes[:, 0] - 0.05, nodes[:, 1] + 0.03)], 1)
    g = np.stack([wl.tg_u(nodes[:, 0], nodes[:, 1]), wl.tg_v(nodes[:, 0], nodes[:, 1])], 1)
    res = roundtrip(orc, f, g)
    # w.r.t. the mesh input: the loss is quadratic in f, so central
    # differences are exact up to rounding
    rng = np.random.default_rng(12)
    d = 1e-6
    for k in rng.choice(mesh.n_nodes, 10, replace=False):
        for ch in range(2):
            fp, fm = f.copy(), f.copy()
            fp[k, ch] += d
            fm[k, ch] -= d
            lp = roundtrip_loss(orc, fp, g)
            lm = roundtrip_loss(orc, fm, g)
            assert abs((lp - lm) / (2 * d) - res["grad_mesh"][k, ch]) < 1e-8
    # w.r.t. particle values (intermediate a = M2P f): dL/da = W^t resid
    W, _ = orc.matrix()
    assert np.allclose(res["grad_vals"], W.T @ res["resid"], atol=1e-14)
    # w.r.t. positions through both operators
    W0, pat0, cl0 = _structure(orc)
    used = 0
    for mu in rng.choice(c.N, 30, replace=False):
        for k in range(2):
            pp, pm = c.pos.copy(), c.pos.copy()
            pp[mu, k] += d
            pm[mu, k] -= d
            op, om = P2MOracle(pp, mesh, c.h), P2MOracle(pm, mesh, c.h)
            if (_structure(op)[1] != pat0).nnz or (_structure(om)[1] != pat0).nnz:
                continue
            fd = (roundtrip_loss(op, f, g) - roundtrip_loss(om, f, g)) / (2 * d)
            assert abs(fd - res["grad_pos"][mu, k]) <= 1e-6 * max(1.0, abs(fd))
            used += 1
    assert used >= 40


def roundtrip_loss(orc, f, g):
    a = m2p(orc.mesh, f, orc.pos)
    W, _ = orc.matrix()
    r = W @ a - g
    return 0.5 * float((r * r).sum())
