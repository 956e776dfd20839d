"""Pins of the oracle's gather (App. A.3.3) and relativistic Boris mover
(App. A.3.3, eq. mover) against closed forms."""
import numpy as np
import pytest


def _coords(dims):
    i, j, k = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    return [a.transpose(2, 1, 0).reshape(-1).astype(float) for a in (i, j, k)]


E_POS = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5]])
B_POS = np.array([[0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])


def _field(dims, pos, f):
    X = _coords(dims)
    return np.concatenate([f(c, [X[a] + pos[c][a] for a in range(3)]) for c in range(3)])


def test_gather_constant_field_is_exact(orc):
    dims = (5, 4, 6)
    e = _field(dims, E_POS, lambda c, r: np.full_like(r[0], [0.3, -1.2, 2.5][c]))
    b = _field(dims, B_POS, lambda c, r: np.full_like(r[0], [-0.7, 0.1, 4.0][c]))
    rng = np.random.default_rng(1)
    for _ in range(50):
        x = rng.uniform(0, 1, 3) * np.array(dims)
        E, B = orc.gather(dims, e, b, x)
        assert np.allclose(E, [0.3, -1.2, 2.5], rtol=0, atol=1e-14)
        assert np.allclose(B, [-0.7, 0.1, 4.0], rtol=0, atol=1e-14)


def test_gather_linear_field_is_exact(orc):
    # node averages of a linear field are the field at the node, and trilinear
    # weighting reproduces a linear function: any stagger mistake shifts it.
    dims = (12, 12, 12)
    A = np.array([[0.1, 0.2, -0.3], [0.05, -0.1, 0.2], [-0.2, 0.15, 0.07]])
    a0 = np.array([1.0, -2.0, 0.5])
    e = _field(dims, E_POS, lambda c, r: a0[c] + sum(A[c][q] * r[q] for q in range(3)))
    b = _field(dims, B_POS, lambda c, r: -a0[c] + sum(A[q][c] * r[q] for q in range(3)))
    rng = np.random.default_rng(2)
    for _ in range(50):
        x = rng.uniform(3, 8, 3)   # away from the periodic seam
        E, B = orc.gather(dims, e, b, x)
        assert np.allclose(E, a0 + A @ x, rtol=0, atol=1e-12)
        assert np.allclose(B, -a0 + A.T @ x, rtol=0, atol=1e-12)


def test_gather_quadratic_field_offset(orc):
    # e_x = x^2 on the e_x edges: node value (x-1/2)^2/2 + (x+1/2)^2/2 = i^2 + 1/4,
    # trilinear in x gives x^2 + d(1-d) + 1/4 with d the in-cell offset.
    dims = (12, 4, 4)
    e = _field(dims, E_POS, lambda c, r: r[0] ** 2 if c == 0 else 0 * r[0])
    b = _field(dims, B_POS, lambda c, r: r[0] ** 2 if c == 2 else 0 * r[0])
    for x0 in [3.0, 3.25, 4.5, 6.9, 7.999]:
        x = np.array([x0, 1.3, 2.7])
        d = x0 - np.floor(x0)
        E, B = orc.gather(dims, e, b, x)
        assert abs(E[0] - (x0 ** 2 + d * (1 - d) + 0.25)) < 1e-12
        assert abs(B[2] - (x0 ** 2 + d * (1 - d) + 0.25)) < 1e-12


def test_boris_pure_b_rotation_angle_and_norm(orc):
    # pure b: |u| is conserved and u turns by 2 arctan|t| per step, clockwise
    # about b for k > 0 (du/dt = k u x b / gamma).
    k, dt = -1.0, 0.5
    B = np.array([0.0, 0.0, 0.8])
    u0 = np.array([0.6, 0.0, 0.3])
    gam = np.sqrt(1 + u0 @ u0)
    t = 0.5 * k * dt * B[2] / gam
    theta = 2 * np.arctan(t)      # signed: rotation by -theta about z
    u = u0.copy()
    n = 200
    for _ in range(n):
        u = orc.boris(k, dt, np.zeros(3), B, u)
    ang = -theta * n
    ref = np.array([u0[0] * np.cos(ang) - u0[1] * np.sin(ang),
                    u0[0] * np.sin(ang) + u0[1] * np.cos(ang), u0[2]])
    assert np.allclose(u, ref, rtol=0, atol=1e-12)
    assert abs(np.linalg.norm(u) - np.linalg.norm(u0)) < 1e-13
    # omega_c dt = 0.2 at gamma = 1 gives a turn of 0.1993373 per step
    assert abs(2 * np.arctan(0.1) - 0.1993373) < 1e-7


def test_boris_larmor_orbit_radius(orc):
    # positions lie on a circle of radius r_L sqrt(1 + |t|^2), r_L = u_perp / (|k| b)
    k, dt = 1.0, 0.5
    B = np.array([0.0, 0.0, 0.5])
    u = np.array([0.0, 0.9, 0.0])
    gam = np.sqrt(1 + u @ u)
    t = 0.5 * k * dt * B[2] / gam
    R = 0.9 / (k * B[2]) * np.sqrt(1 + t * t)
    x = np.zeros(3)
    pts = []
    for _ in range(300):
        u = orc.boris(k, dt, np.zeros(3), B, u)
        x = x + dt * u / np.sqrt(1 + u @ u)
        pts.append(x[:2].copy())
    P = np.array(pts)
    # circle fit: centre is the mean over whole turns; check radius spread
    Amat = np.c_[2 * P, np.ones(len(P))]
    sol = np.linalg.lstsq(Amat, (P ** 2).sum(1), rcond=None)[0]
    c = sol[:2]
    r = np.sqrt(((P - c) ** 2).sum(1))
    assert np.max(np.abs(r - R)) < 1e-10


def test_boris_pure_e_is_linear(orc):
    k, dt = -1.0 / 25.0, 0.5
    E = np.array([0.01, -0.02, 0.005])
    u = np.array([0.1, 0.2, -0.3])
    u1 = u.copy()
    for _ in range(100):
        u1 = orc.boris(k, dt, E, np.zeros(3), u1)
    assert np.allclose(u1, u + 100 * k * dt * E, rtol=0, atol=1e-13)


def test_boris_exb_drift(orc):
    # average velocity -> e x b / b^2 for |e| << |b| (to O((w_c dt)^2) and the
    # residual gyration over the window)
    k, dt = -1.0, 0.5
    E = np.array([0.02, 0.0, 0.0])
    B = np.array([0.0, 0.0, 0.4])
    vd = np.cross(E, B) / (B @ B)
    u = np.zeros(3)
    x = np.zeros(3)
    n = 20000
    for _ in range(n):
        u = orc.boris(k, dt, E, B, u)
        x = x + dt * u / np.sqrt(1 + u @ u)
    v = x / (n * dt)
    assert abs(v[1] - vd[1]) < 2e-3 * abs(vd[1])
    assert abs(v[0]) < 2e-3 * abs(vd[1])


@pytest.mark.parametrize("reverse", [False, True])
def test_boris_is_time_reversible(orc, reverse):
    rng = np.random.default_rng(3)
    E = rng.normal(size=3) * 0.1
    B = rng.normal(size=3) * 0.5
    u0 = rng.normal(size=3)
    k = -1.0 if reverse else 1.0 / 25
    u1 = orc.boris(k, 0.5, E, B, u0)
    u2 = orc.boris(k, -0.5, E, B, u1)
    assert np.allclose(u2, u0, rtol=0, atol=1e-13)
