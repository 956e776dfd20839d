"""Whole-loop pins of the oracle (App. A.3.1): cold plasma modes against closed
forms and the printed theory columns of Table 1, Gauss's law kept to roundoff by
the charge-conserving scheme (Sect. 2.1, App. A.1), and energy bookkeeping."""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _lattice(dims, sub):
    i, j, k = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    base = np.stack([i.ravel(), j.ravel(), k.ravel()], 1).astype(float)
    return base + np.asarray(sub)


def _freq_single(s, dt):
    """one pure sinusoid: s[n+1] + s[n-1] = 2 cos(w dt) s[n]"""
    s = np.asarray(s)
    c = np.sum(s[1:-1] * (s[2:] + s[:-2])) / (2 * np.sum(s[1:-1] ** 2))
    return np.arccos(c) / dt


def _freqs_prony(s, dt, nmodes):
    """frequencies of a sum of nmodes undamped real sinusoids (linear prediction)"""
    s = np.asarray(s)
    p = 2 * nmodes
    A = np.array([s[n - p:n][::-1] for n in range(p, len(s))])
    coef = np.linalg.lstsq(A, s[p:], rcond=None)[0]
    roots = np.roots(np.r_[1.0, -coef])
    w = np.sort(np.abs(np.angle(roots)))[::2] / dt
    return w


def test_cold_pair_oscillation_discrete_dispersion(orc):
    # k = 0 Langmuir oscillation of a cold pair plasma: leap-frog gives
    # sin(w dt/2) = w_P dt/2 with w_P = sqrt(2)/n_x (Sect. 3.1, m_i = m_e)
    dims, n_x, dt, u0 = (2, 2, 2), 10.0, 0.5, 1e-4
    st = orc.State(dims, dt, n_x=n_x, rho0=2, species=[(-1, 1), (1, 1)])
    x = _lattice(dims, [0.3, 0.6, 0.45])
    st.add_particles(0, x, np.tile([u0, 0, 0], (len(x), 1)))
    st.add_particles(1, x, np.tile([-u0, 0, 0], (len(x), 1)))
    s = []
    for _ in range(400):
        st.step(1)
        s.append(st.u[st.species == 0, 0].sum())
    w = _freq_single(s, dt)
    w_ref = 2 * np.arcsin(np.sqrt(2) / n_x * dt / 2) / dt
    assert abs(w_ref - 0.14145084) < 1e-8
    assert abs(w - w_ref) < 1e-7 * w_ref


def test_langmuir_mass_ratio_49_matches_table1(orc):
    gold = json.load(open(os.path.join(GOLD, "table1_cold_modes.json")))
    mi = gold["mi_over_me_for_omega_P"]
    dims, n_x, dt, u0 = (2, 2, 2), 10.0, 0.25, 1e-4
    st = orc.State(dims, dt, n_x=n_x, rho0=2, species=[(-1, 1), (1, mi)])
    x = _lattice(dims, [0.7, 0.2, 0.5])
    st.add_particles(0, x, np.tile([0, u0, 0], (len(x), 1)))
    st.add_particles(1, x, np.zeros((len(x), 3)))
    s = []
    for _ in range(1500):
        st.step(1)
        s.append(st.u[st.species == 0, 1].sum())
    # the centre of mass drifts: difference the series to drop the constant
    w = _freq_single(np.diff(s), dt) * n_x  # in units of omega_pe = 1/n_x
    w_disc = 2 * np.arcsin(np.sqrt(1 + 1.0 / mi) / n_x * dt / 2) / dt * n_x
    assert abs(w - w_disc) < 1e-6
    assert abs(w - gold["omega_P"]) < 0.5 * gold["spectral_resolution"]


@pytest.mark.parametrize("row", range(4))
def test_magnetized_cold_modes_match_table1(orc, row):
    # electrons on immobile ions in a uniform b along z: the k = 0 transverse
    # momentum oscillates at omega_L and omega_R (Sect. 3.1.2, Table 1)
    gold = json.load(open(os.path.join(GOLD, "table1_cold_modes.json")))["rows"][row]
    dims, n_x, dt, u0 = (2, 2, 2), 10.0, 0.25, 1e-4
    st = orc.State(dims, dt, n_x=n_x, rho0=2, species=[(-1, 1), (1, 1e12)])
    x = _lattice(dims, [0.4, 0.55, 0.35])
    st.add_particles(0, x, np.tile([u0, 0, 0], (len(x), 1)))
    st.add_particles(1, x, np.zeros((len(x), 3)))
    n = st.n
    st.b[2 * n:] = gold["omega_ce"] / n_x
    s = []
    for _ in range(3000):
        st.step(1)
        s.append(st.u[st.species == 0, 0].sum())
    wL, wR = _freqs_prony(s, dt, 2) * n_x
    wce = gold["omega_ce"]
    assert abs(wL - 0.5 * (np.sqrt(wce ** 2 + 4) - wce)) < 5e-3
    assert abs(wR - 0.5 * (np.sqrt(wce ** 2 + 4) + wce)) < 5e-3
    assert abs(wL - gold["omega_L"]) < 0.01
    assert abs(wR - gold["omega_R"]) < 0.01


def _thermal(orc, dims, ppc, theta, seed, n_x=10.0):
    npairs = ppc * int(np.prod(dims))
    st = orc.State(dims, 0.5, n_x=n_x, rho0=2 * ppc, species=[(-1, 1), (1, 1)])
    sp = {"theta": theta, "gb": 0.0, "axis": 1}
    x, ua, ub = orc.load_pairs(dims, seed, 0, npairs, sp, sp)
    st.add_particles(0, x, ua)
    st.add_particles(1, x, ub)
    st.backward_half()
    return st


def test_gauss_law_kept_to_roundoff(orc):
    st = _thermal(orc, (6, 5, 4), 4, 0.1, seed=7)
    d0 = st.diag()
    assert d0["gauss_max"] < 1e-15
    st.step(40)
    d1 = st.diag()
    rho_scale = st.alpha0 * 4
    assert d1["gauss_max"] < 1e-12 * rho_scale
    # the field did respond to the plasma
    assert d1["W_E"].sum() > 1e-6 * d1["K"].sum()


def test_energy_bookkeeping_short_run(orc):
    # total energy (1/alpha0) sum e^2/2 + b^2/2 + sum (m/m_e)(gamma-1) is
    # conserved up to the scheme's self-heating; a wrong alpha, k or field
    # time level shows up as an O(1) exchange imbalance.
    st = _thermal(orc, (6, 6, 6), 8, 0.1, seed=3)
    d0 = st.diag()
    E0 = d0["W_E"].sum() + d0["W_B"].sum() + d0["K"].sum()
    st.step(60)
    d1 = st.diag()
    E1 = d1["W_E"].sum() + d1["W_B"].sum() + d1["K"].sum()
    assert d1["W_E"].sum() > 1e-4 * E0        # fields took a share
    assert abs(E1 - E0) / E0 < 2e-3


def test_backward_half_step_reverses_push(orc):
    dims = (4, 4, 4)
    rng = np.random.default_rng(5)
    st = orc.State(dims, 0.5, n_x=10, rho0=2, species=[(-1, 1)])
    st.b[:] = rng.normal(size=st.b.shape) * 0.1
    st.e[:] = rng.normal(size=st.e.shape) * 0.05
    x = rng.uniform(0, 4, (20, 3))
    u = rng.normal(size=(20, 3))
    st.add_particles(0, x, u)
    b0 = st.b.copy()
    st.backward_half()
    # b^{-dt/2} = b^0 + (dt/2) curl e^0
    assert np.allclose(st.b, b0 + 0.25 * orc.curl_e(dims, st.e), atol=1e-15)
    # pushing u^{-dt/2} forward by dt/2 in the same t=0 fields recovers u^0
    for p in range(20):
        E, B = orc.gather(dims, st.e, b0, x[p])
        assert np.allclose(orc.boris(-1.0, 0.25, E, B, st.u[p]), u[p], atol=1e-13)
