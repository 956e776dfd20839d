"""Pins of the oracle's Yee field update (App. A.3.2) against closed forms.

A discrete plane wave is an exact eigenvector of the staggered leap-frog curl
scheme: with kappa_c = 2 sin(k_c/2), the fields rotate by omega*dt per step with
sin(omega dt/2) = (dt/2)|kappa| and b_hat = dt kappa x e_hat / (2 sin(omega dt/2)).
A sign error, a swapped stagger offset or a wrong time level in any curl term
breaks the agreement at the first step.
"""
import numpy as np
import pytest

E_POS = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5]])
B_POS = np.array([[0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])


def _coords(dims):
    i, j, k = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    # flatten with x fastest: index i + nx*(j + ny*k)
    return [a.transpose(2, 1, 0).reshape(-1).astype(float) for a in (i, j, k)]


def _mode(dims, m, e_dir, dt, n_e, n_b):
    kv = 2 * np.pi * np.array(m, float) / np.array(dims, float)
    kap = 2 * np.sin(kv / 2)
    e_hat = np.array(e_dir, float)
    assert abs(np.dot(kap, e_hat)) < 1e-14
    s = 0.5 * dt * np.linalg.norm(kap)
    om = 2 * np.arcsin(s) / dt
    b_hat = dt * np.cross(kap, e_hat) / (2 * s)
    X = _coords(dims)
    e = np.concatenate([e_hat[c] * np.cos(sum(kv[a] * (X[a] + E_POS[c][a]) for a in range(3))
                                          - om * n_e * dt) for c in range(3)])
    b = np.concatenate([b_hat[c] * np.cos(sum(kv[a] * (X[a] + B_POS[c][a]) for a in range(3))
                                          - om * n_b * dt) for c in range(3)])
    return e, b, om


@pytest.mark.parametrize("dims,m,e_dir", [
    ((16, 4, 4), (1, 0, 0), (0, 1, 0)),
    ((16, 4, 4), (3, 0, 0), (0, 0, 1)),
    ((4, 12, 4), (0, 2, 0), (1, 0, 0)),
    ((4, 4, 10), (0, 0, 1), (0, 1, 0)),
    ((8, 8, 4), (1, 2, 0), (0, 0, 1)),
])
def test_plane_wave_eigenmode(orc, dims, m, e_dir):
    dt = 0.5
    st = orc.State(dims, dt, n_x=10, rho0=1, species=[(-1, 1)])
    st.e, st.b, om = _mode(dims, m, e_dir, dt, 0.0, -0.5)
    nsteps = 37
    st.step(nsteps)
    e_ref, b_ref, _ = _mode(dims, m, e_dir, dt, nsteps, nsteps - 0.5)
    assert np.max(np.abs(st.e - e_ref)) < 1e-12
    assert np.max(np.abs(st.b - b_ref)) < 1e-12


def test_oblique_3d_mode(orc):
    dims = (8, 6, 10)
    m = (1, 1, 2)
    kv = 2 * np.pi * np.array(m) / np.array(dims)
    kap = 2 * np.sin(kv / 2)
    e_dir = np.cross(kap, [1.0, 0.0, 0.0])
    e_dir /= np.linalg.norm(e_dir)
    dt = 0.45
    st = orc.State(dims, dt, n_x=10, rho0=1, species=[(-1, 1)])
    st.e, st.b, om = _mode(dims, m, e_dir, dt, 0.0, -0.5)
    st.step(25)
    e_ref, b_ref, _ = _mode(dims, m, e_dir, dt, 25, 24.5)
    assert np.max(np.abs(st.e - e_ref)) < 1e-12
    assert np.max(np.abs(st.b - b_ref)) < 1e-12


def test_dispersion_value_1d():
    # k = 2 pi / 16, dt = 0.5: sin(w dt/2) = dt sin(k/2); continuum w = k
    k = 2 * np.pi / 16
    w = 2 * np.arcsin(0.5 * np.sin(k / 2)) / 0.5
    assert abs(w - 0.390802) < 1e-6
    assert abs(k - 0.392699) < 1e-6


def test_curl_of_gradient_vanishes(orc):
    # discrete identity curl(grad phi) = 0 for e = grad phi on the edges
    dims = (5, 6, 7)
    rng = np.random.default_rng(0)
    phi = rng.standard_normal(dims[::-1]).reshape(-1)  # node values, x fastest
    P = phi.reshape(dims[2], dims[1], dims[0])
    ex = (np.roll(P, -1, axis=2) - P).reshape(-1)
    ey = (np.roll(P, -1, axis=1) - P).reshape(-1)
    ez = (np.roll(P, -1, axis=0) - P).reshape(-1)
    c = orc.curl_e(dims, np.concatenate([ex, ey, ez]))
    assert np.max(np.abs(c)) < 1e-13
    # and div(curl b) = 0 at the nodes
    b = rng.standard_normal(3 * np.prod(dims))
    cb = orc.curl_b(dims, b)
    n = int(np.prod(dims))
    X = cb[:n].reshape(P.shape)
    Y = cb[n:2 * n].reshape(P.shape)
    Z = cb[2 * n:].reshape(P.shape)
    div = (X - np.roll(X, 1, axis=2)) + (Y - np.roll(Y, 1, axis=1)) + (Z - np.roll(Z, 1, axis=0))
    assert np.max(np.abs(div)) < 1e-12
