"""Pins of the oracle's fourth-order field solver (App. A.3.2, last paragraph;
App. B, third item): Faraday's law with the staggered fourth-order curl, Ampere's
law with the Yee curl (reading stated in pic_oracle.c).

* The stencil is fourth-order accurate: the curl of a smooth field converges
  to the analytic derivative as h^4 (the Yee curl as h^2).
* A discrete plane wave is an exact eigenvector of the mixed scheme: with
  kappa_a = 2 sin(k_a/2) and kappa4_a = (9/4) sin(k_a/2) - (1/12) sin(3 k_a/2),
  the fields rotate by omega dt per step with
  sin^2(omega dt / 2) = (dt/2)^2 kappa . kappa4 = (dt/2)^2 sum_a [4 s_a^2 + (2/3) s_a^4],
  s_a = sin(k_a/2), e perpendicular to kappa and
  b_hat = dt kappa4 x e_hat / (2 sin(omega dt/2)).
* The fourth-order divergence of b is kept (div4 curl4 = 0), and Gauss's law
  for e with the second-order divergence holds to roundoff in a plasma,
  because Ampere's law is unchanged.
* Its phase velocity is closer to c than Yee's, on the axes and at 45 degrees.
"""
import numpy as np
import pytest

E_POS = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5]])
B_POS = np.array([[0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])


def _coords(dims):
    i, j, k = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    return [a.transpose(2, 1, 0).reshape(-1).astype(float) for a in (i, j, k)]


def _kappas(kv):
    return 2 * np.sin(kv / 2), 2.25 * np.sin(kv / 2) - np.sin(1.5 * kv) / 12


def _mode(dims, m, e_dir, dt, n_e, n_b):
    kv = 2 * np.pi * np.array(m, float) / np.array(dims, float)
    kap, kap4 = _kappas(kv)
    e_hat = np.array(e_dir, float)
    assert abs(np.dot(kap, e_hat)) < 1e-14
    s = 0.5 * dt * np.sqrt(np.dot(kap, kap4))
    om = 2 * np.arcsin(s) / dt
    b_hat = dt * np.cross(kap4, e_hat) / (2 * s)
    X = _coords(dims)
    e = np.concatenate([e_hat[c] * np.cos(sum(kv[a] * (X[a] + E_POS[c][a]) for a in range(3))
                                          - om * n_e * dt) for c in range(3)])
    b = np.concatenate([b_hat[c] * np.cos(sum(kv[a] * (X[a] + B_POS[c][a]) for a in range(3))
                                          - om * n_b * dt) for c in range(3)])
    return e, b, om


def _state(orc, dims, dt):
    st = orc.State(dims, dt, n_x=10, rho0=1, species=[(-1, 1)])
    st.faraday4 = True
    return st


@pytest.mark.parametrize("dims,m,e_dir", [
    ((16, 4, 4), (1, 0, 0), (0, 1, 0)),
    ((16, 4, 4), (5, 0, 0), (0, 0, 1)),
    ((4, 12, 4), (0, 2, 0), (1, 0, 0)),
    ((4, 4, 10), (0, 0, 3), (0, 1, 0)),
    ((8, 8, 4), (1, 2, 0), (0, 0, 1)),
])
def test_plane_wave_eigenmode_fourth_order_faraday(orc, dims, m, e_dir):
    dt = 0.5
    st = _state(orc, dims, dt)
    st.e, st.b, om = _mode(dims, m, e_dir, dt, 0.0, -0.5)
    st.step(37)
    e_ref, b_ref, _ = _mode(dims, m, e_dir, dt, 37, 36.5)
    assert np.max(np.abs(st.e - e_ref)) < 1e-12
    assert np.max(np.abs(st.b - b_ref)) < 1e-12


def test_oblique_3d_mode_fourth_order_faraday(orc):
    dims, m, dt = (8, 6, 10), (1, 1, 2), 0.5
    kv = 2 * np.pi * np.array(m) / np.array(dims)
    kap, _ = _kappas(kv)
    e_dir = np.cross(kap, [1.0, 0.0, 0.0])
    e_dir /= np.linalg.norm(e_dir)
    st = _state(orc, dims, dt)
    st.e, st.b, _ = _mode(dims, m, e_dir, dt, 0.0, -0.5)
    st.step(25)
    e_ref, b_ref, _ = _mode(dims, m, e_dir, dt, 25, 24.5)
    assert np.max(np.abs(st.e - e_ref)) < 1e-12
    assert np.max(np.abs(st.b - b_ref)) < 1e-12
    # the same mode under Yee rotates by another angle: the test tells them apart
    y = orc.State(dims, dt, n_x=10, rho0=1, species=[(-1, 1)])
    y.e, y.b, _ = _mode(dims, m, e_dir, dt, 0.0, -0.5)
    y.step(25)
    assert np.max(np.abs(y.e - e_ref)) > 1e-3


def test_curl4_converges_at_fourth_order(orc):
    # e_z = sin(2 pi y / N) on the e_z edges: (curl e)_x = d_y e_z at the b_x
    # positions (i, j + 1/2, k + 1/2) is (2 pi / N) cos(2 pi (j + 1/2) / N)
    errs4, errs2 = [], []
    for N in (16, 32, 64):
        dims = (2, N, 2)
        X = _coords(dims)
        n = int(np.prod(dims))
        e = np.zeros(3 * n)
        e[2 * n:] = np.sin(2 * np.pi * X[1] / N)
        exact = 2 * np.pi / N * np.cos(2 * np.pi * (X[1] + 0.5) / N)
        # derivative per cell; scale by N to compare slopes of the continuum field
        errs4.append(np.max(np.abs(orc.curl_e4(dims, e)[:n] - exact)) * N)
        errs2.append(np.max(np.abs(orc.curl_e(dims, e)[:n] - exact)) * N)
    r4 = [errs4[i] / errs4[i + 1] for i in range(2)]
    r2 = [errs2[i] / errs2[i + 1] for i in range(2)]
    assert all(15.0 < r < 17.0 for r in r4), r4
    assert all(3.8 < r < 4.2 for r in r2), r2


def test_fourth_order_divergence_of_curl4_vanishes(orc):
    # Faraday with curl4 keeps div4 b: div4(curl4 e) = 0 for any e, where
    # div4 uses the same fourth-order differences (at the cell centres);
    # the second-order divergence does not vanish (the identity is the
    # solver's own)
    dims = (7, 6, 8)
    rng = np.random.default_rng(3)
    e = rng.standard_normal(3 * np.prod(dims))
    c = orc.curl_e4(dims, e)
    n = int(np.prod(dims))
    F = [c[q * n:(q + 1) * n].reshape(dims[2], dims[1], dims[0]) for q in range(3)]
    ax = {0: 2, 1: 1, 2: 0}     # array axis of each grid axis (x fastest)

    # b_c sits half a cell below the cell centre (i+1/2, j+1/2, k+1/2) along
    # c: the differences are taken there, from index i (and i-1, i+1, i+2)
    def d4(f, a):
        A = ax[a]
        return 9 / 8 * (np.roll(f, -1, A) - f) - 1 / 24 * (np.roll(f, -2, A) - np.roll(f, 1, A))

    def d2(f, a):
        return np.roll(f, -1, ax[a]) - f
    div4 = d4(F[0], 0) + d4(F[1], 1) + d4(F[2], 2)
    div2 = d2(F[0], 0) + d2(F[1], 1) + d2(F[2], 2)
    assert np.max(np.abs(div4)) < 1e-12
    assert np.max(np.abs(div2)) > 1e-3


def test_gauss_law_kept_with_fourth_order_faraday(orc):
    # a hot pair plasma: Ampere's curl is still Yee's, so div2 e - rho stays
    # at roundoff over 100 steps
    dims, ppc, dt = (6, 5, 4), 4, 0.5
    st = orc.State(dims, dt, n_x=10.0, rho0=2 * ppc, species=[(-1, 1), (1, 1)])
    st.faraday4 = True
    sp = {"theta": 0.3, "gb": 0.0, "axis": 1}
    x, ua, ub = orc.load_pairs(dims, 5, 0, ppc * int(np.prod(dims)), sp, sp)
    st.add_particles(0, x, ua)
    st.add_particles(1, x, ub)
    st.backward_half()
    st.step(100)
    d = st.diag()
    assert d["gauss_max"] < 1e-12 * st.alpha0 * ppc
    assert d["W_E"].sum() > 1e-6 * d["K"].sum()


def test_phase_velocity_closer_to_c_than_yee():
    # closed forms of the two dispersion relations at dt = 0.5, for k of 4
    # and 8 cells per wavelength along an axis and at 45 degrees in a plane
    dt = 0.5
    for lam in (8.0, 4.0):
        for direction in ((1.0, 0.0, 0.0), (1 / np.sqrt(2), 1 / np.sqrt(2), 0.0)):
            kv = 2 * np.pi / lam * np.array(direction)
            kap, kap4 = _kappas(kv)
            w_yee = 2 * np.arcsin(0.5 * dt * np.linalg.norm(kap)) / dt
            w_4 = 2 * np.arcsin(0.5 * dt * np.sqrt(kap @ kap4)) / dt
            k = np.linalg.norm(kv)
            assert abs(w_4 / k - 1) < abs(w_yee / k - 1)
    # the mixed scheme's Courant bound: (dt/2)^2 max sum_a (4 s^2 + 2/3 s^4) = 1
    # gives dt < 2 / sqrt(14) in 3-D
    assert abs(2 / np.sqrt(3 * (4 + 2 / 3)) - 0.534522) < 1e-6
