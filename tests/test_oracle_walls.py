"""Pins of the oracle's perfectly conducting walls (App. A.4): a standing
wave between two walls follows the closed form of the discrete scheme (and
fails without the wall condition for an odd mode), particles bounce off the
walls in straight lines, and Gauss's law holds in the interior of a thermal
plasma bouncing between walls."""
import numpy as np
import pytest


def _standing_wave(n, m, dt, steps):
    k = np.pi * m / n
    om = 2 * np.arcsin(dt * np.sin(k / 2)) / dt          # sin(om dt/2) = dt sin(k/2)
    B = -dt * np.sin(k / 2) / np.sin(om * dt / 2)
    i = np.arange(n)
    e_y = lambda t: np.sin(k * i) * np.cos(om * t)                 # at (i, j+1/2, k)
    b_z = lambda t: B * np.cos(k * (i + 0.5)) * np.sin(om * t)     # at (i+1/2, j+1/2, k)
    return e_y, b_z


def test_standing_wave_between_walls(orc):
    n, m, dt, steps = 16, 3, 0.5, 40
    dims = (n, 1, 1)
    e_y, b_z = _standing_wave(n, m, dt, steps)
    for wall, tol in ((0, 1e-12), (-1, None)):
        st = orc.State(dims, dt, 10.0, 1.0, [(-1.0, 1.0)])
        st.wall = wall
        st.e[n:2 * n] = e_y(0.0)
        st.b[2 * n:3 * n] = b_z(-0.5 * dt)
        st.step(steps)
        err = max(np.abs(st.e[n:2 * n] - e_y(steps * dt)).max(), np.abs(st.b[2 * n:3 * n] - b_z((steps - 0.5) * dt)).max())
        if tol is not None:
            assert err < tol, err
            assert np.abs(st.e[:n]).max() == 0 and np.abs(st.e[2 * n:]).max() == 0
        else:
            assert err > 1e-2        # an odd mode is not periodic: the wall condition is what holds it


@pytest.mark.parametrize("w", [0, 1, 2])
def test_particles_bounce_off_the_walls(orc, w):
    # a co-located electron-positron pair deposits no net current, so the fields
    # stay zero and both move in straight lines between bounces
    dt = 0.5
    dims = [4, 4, 4]
    dims[w] = 6
    st = orc.State(tuple(dims), dt, 10.0, 2.0, [(-1.0, 1.0), (1.0, 1.0)])
    st.wall = w
    perm = [(w + k) % 3 for k in range(3)]          # the wall axis takes the role of x
    x0 = np.zeros((2, 3))
    u0 = np.zeros((2, 3))
    x0[:, perm] = [[0.3, 1.5, 2.5], [5.6, 0.5, 3.9]]
    u0[:, perm] = [[-0.9, 0.2, 0.0], [0.7, -0.3, 0.4]]
    st.add_particles(0, x0, u0)
    st.add_particles(1, x0, u0)
    steps = 23
    st.step(steps)
    for p in range(2):
        v = u0[p] / np.sqrt(1 + u0[p] @ u0[p])
        x = x0[p] + steps * dt * v
        L = dims[w]
        # unfold the bounces along the wall axis: reflect into [0, L)
        xx = np.mod(x[w], 2 * L)
        want_x = np.mod(x, dims)
        want_x[w] = xx if xx < L else 2 * L - xx
        sgn = 1.0 if xx < L else -1.0
        for s in range(2):
            got = st.x[st.species == s][p]
            assert np.abs(got - want_x).max() < 1e-12, (got, want_x)
            assert abs(st.u[st.species == s][p][w] - sgn * u0[p][w]) < 1e-14
    assert np.abs(st.e).max() < 1e-15 and np.abs(st.b).max() < 1e-15


@pytest.mark.parametrize("w", [0, 1, 2])
def test_gauss_law_in_the_interior_with_walls(orc, w):
    dims = [6, 6, 6]
    dims[w] = 8
    ppc = 6
    rng = np.random.default_rng(4 + w)
    st = orc.State(tuple(dims), 0.5, 10.0, 2 * ppc, [(-1.0, 1.0), (1.0, 1.0)])
    st.wall = w
    npairs = ppc * int(np.prod(dims))
    x = rng.uniform(0, 1, (npairs, 3)) * np.array(dims)
    st.add_particles(0, x, 0.5 * rng.standard_normal((npairs, 3)))
    st.add_particles(1, x, 0.5 * rng.standard_normal((npairs, 3)))
    st.step(30)
    d = st.diag()
    assert d["gauss_max"] < 1e-12, d["gauss_max"]
    assert int(d["count"].sum()) == 2 * npairs
    assert np.all((st.x[:, w] >= 0) & (st.x[:, w] < dims[w]))
    # the walls keep tangential e and normal b at zero on their plane
    n = int(np.prod(dims))
    idx = np.arange(n)
    coord = [idx % dims[0], (idx // dims[0]) % dims[1], idx // (dims[0] * dims[1])]
    wallp = coord[w] == 0
    for c in range(3):
        f = st.b if c == w else st.e
        assert np.all(f[c * n:(c + 1) * n][wallp] == 0)
