"""Pins of the oracle's Maxwell-Juttner loader (Sect. 4, App. D), its Philox
generator and the relativistic Harris relations (App. C).

Moments are checked against the closed forms of the table of averages
(tab:averages_Juttner, Sect. 4.3; the <beta^2> row is not used, it exceeds 1 at
Theta = 1), and against the printed parameters of Fig. testJuttner
(T = m c^2, Gamma0 beta0 = sqrt 2, 10^6 particles).
"""
import json
import os

import numpy as np
import pytest
from scipy import integrate, special

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((5, 7, 0, 0), (123, 456)),
    ((2 ** 63, 1, 2, 3), (2 ** 64 - 1, 99)),
    ((12345678901, 2, 0, 0), (1, 0)),
])
def test_philox_matches_numpy(orc, ctr, key):
    # numpy's Philox bit generator is Philox-4x64-10; it increments its 256-bit
    # counter before producing a block, so start it one below.
    c = sum(int(v) << (64 * i) for i, v in enumerate(ctr))
    bg = np.random.Philox(counter=(c - 1) % (1 << 256), key=sum(int(v) << (64 * i) for i, v in enumerate(key)))
    ref = bg.random_raw(4)
    got = orc.philox4x64(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64))
    assert np.array_equal(got, ref)


def _kappa32(mu):
    return special.kve(3, mu) / special.kve(2, mu)


def _jY(y, mu, G, beta0):
    # App. D, eq. distr_y, normalised with K_2 (scaled Bessel to avoid underflow)
    gy = np.sqrt(1 + y * y)
    return (1 + mu * G * gy) / (2 * mu * G ** 3 * special.kve(2, mu)) * np.exp(
        -mu * G * (gy - beta0 * y) + mu)


@pytest.mark.parametrize("theta,gb", [(0.1, 0.0), (1.0, np.sqrt(2)), (0.01, np.sqrt(8.0))])
def test_table_quantiles(orc, theta, gb):
    mu = 1 / theta
    G = np.sqrt(1 + gb * gb)
    beta0 = gb / G
    N = 1 << 12
    tab = orc.mj_table(theta, gb, N=N)
    lo, hi = orc.mj_range(mu, beta0)
    assert tab[0] == lo and tab[-1] == hi
    assert np.all(np.diff(tab) > 0)
    # the marginal integrates to one with the paper's normalisation
    tot = integrate.quad(_jY, lo, hi, args=(mu, G, beta0), limit=400, epsabs=1e-14, epsrel=1e-13,
                         points=[gb])[0]
    assert abs(tot - 1) < 1e-10
    for i in [1, 7, N // 4, N // 2, 3 * N // 4, N - 3]:
        F = integrate.quad(_jY, lo, tab[i], args=(mu, G, beta0), limit=400, epsabs=1e-14,
                           epsrel=1e-13)[0]
        assert abs(F - i / N) < 1e-10


def test_radial_solve_closed_form(orc):
    rng = np.random.default_rng(0)
    for a in [1.0, 3.7, 10.0, 100.0, 3000.0]:
        for w in rng.uniform(1e-12, 1, 20):
            r = orc.mj_radial(a, w)
            x = a * np.sqrt(1 + r * r)
            # l(x) = w l(a), l(x) = (1 + x) exp(-x), compared in logs
            lhs = np.log1p(x) - x
            rhs = np.log(w) + np.log1p(a) - a
            assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(rhs))
    assert orc.mj_radial(5.0, 1.0) == 0.0


def _sample(orc, theta, gb, axis, n=1_000_000, seed=11):
    dims = (10, 10, 10)
    sp = {"theta": theta, "gb": gb, "axis": axis}
    _, ua, ub = orc.load_pairs(dims, seed, 3, n // 2, sp, sp)
    return np.concatenate([ua, ub])


def _close(samples, ref, nsig=5.0):
    m = samples.mean()
    s = samples.std() / np.sqrt(len(samples))
    assert abs(m - ref) < nsig * s + 1e-12, (m, ref, s)


@pytest.mark.parametrize("theta", [0.05, 0.1, 1.0])
def test_rest_frame_moments(orc, theta):
    u = _sample(orc, theta, 0.0, 1)
    mu = 1 / theta
    g = np.sqrt(1 + (u * u).sum(1))
    _close(g, _kappa32(mu) - theta)                     # <gamma>
    _close((u * u).sum(1), 3 * theta * _kappa32(mu))    # <(gamma beta)^2>
    _close((u * u).sum(1) / g, 3 * theta)               # <gamma beta^2>
    for a in range(3):
        _close(u[:, a], 0.0)
        _close(u[:, a] ** 2 / g, theta)                 # <p_a v_a>


@pytest.mark.parametrize("theta,gb,axis", [
    (1.0, np.sqrt(2.0), 1),     # Fig. testJuttner parameters
    (0.01, np.sqrt(8.0), 0),    # Gamma0 = 3 beam along x
    (1.0, -0.68, 2),            # Harris-sheet drift along -z
    (0.3, 2.0, 0),
])
def test_drifting_moments(orc, theta, gb, axis):
    u = _sample(orc, theta, gb, axis)
    mu = 1 / theta
    G = np.sqrt(1 + gb * gb)
    b0 = gb / G
    k32 = _kappa32(mu)
    g = np.sqrt(1 + (u * u).sum(1))
    _close(g, G * k32 - 1 / (mu * G))                   # <gamma>
    _close(u[:, axis], k32 * G * b0)                    # <gamma v> along the drift
    _close(u[:, axis] / g, b0)                          # <v> = U0
    _close(u[:, axis] ** 2 / g, theta / G + G * b0 ** 2 * k32)   # <p_y v_y>
    for a in range(3):
        if a != axis:
            _close(u[:, a], 0.0)
            _close(u[:, a] ** 2 / g, theta / G)         # <p_x v_x> = Theta/Gamma0
    if axis == 1 and abs(gb - np.sqrt(2)) < 1e-12:
        # numbers quoted for Fig. testJuttner
        assert abs(G * k32 - 1 / (mu * G) - 6.992476) < 1e-6
        assert abs(k32 * G * b0 - 6.180737) < 1e-6


def test_positions_uniform_and_harris(orc):
    dims = (64, 32, 4)
    sp = {"theta": 0.1, "gb": 0.0, "axis": 1}
    x, _, _ = orc.load_pairs(dims, 5, 0, 200_000, sp, sp)
    assert np.all(x >= 0) and np.all(x < np.array(dims))
    for a in range(3):
        _close(x[:, a], dims[a] / 2)
    L, c, h = 6.0, 16.0, 16.0
    x, _, _ = orc.load_pairs(dims, 5, 1, 200_000, sp, sp, profile=1, paxis=0, centre=c, L=L,
                             halfw=h)
    s = x[:, 0] - c
    assert np.all(np.abs(s) <= h)
    # second moment of the truncated sech^2 profile (App. C density n' ~ 1/cosh^2)
    num = integrate.quad(lambda t: t * t / np.cosh(t / L) ** 2, -h, h)[0]
    den = integrate.quad(lambda t: 1 / np.cosh(t / L) ** 2, -h, h)[0]
    _close(s * s, num / den)
    _close(x[:, 1], dims[1] / 2)


def test_harris_relations_reproduce_table4(orc):
    gold = json.load(open(os.path.join(GOLD, "table4_harris.json")))
    for row in gold["rows"]:
        p = orc.harris_params(row["Theta"], row["GammaU_over_c"], chi=1.0, mi_over_me=1.0)
        assert abs(p["wce_over_wpe"] - row["omega_ce_over_omega_pe"]) <= 0.006
        # printed L/d_e for Theta = 0.1 is 0.83 where the relations give 0.8205
        assert abs(p["L_over_de"] - row["L_over_de"]) <= 0.011
        assert abs(p["gu_i"] + row["GammaU_over_c"]) < 1e-15
    # pressure balance (App. C): B0^2/(2 mu0) = n'_e T_e + n'_i T_i, i.e.
    # (w_ce/w'_pe)^2 / 2 = Theta_e (1 + T_i/T_e) in units of n'_e m_e c^2
    for chi, th in [(1.0, 0.3), (1.5, 0.1), (3.0, 1.0)]:
        p = orc.harris_params(th, 0.5, chi=chi, mi_over_me=25.0)
        assert abs(p["wce_over_wpe_prime"] ** 2 / 2 - th * (2 * chi)) < 1e-14
        assert abs(p["theta_i"] - (2 * chi - 1) * th / 25.0) < 1e-15
