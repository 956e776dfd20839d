"""Pins of the oracle's current smoothing (App. A.3.4, last paragraph): the
response to a single value is the printed weight pattern, the sum is kept, the
grid's highest mode is removed, the smoothing commutes with the discrete
divergence, and with it the smoothed charge still satisfies Gauss's law over
a run."""
import numpy as np


def test_single_value_spreads_with_the_printed_weights(orc):
    dims = (7, 6, 5)
    n = int(np.prod(dims))
    f = np.zeros(n)
    i0, j0, k0 = 3, 2, 2
    f[i0 + dims[0] * (j0 + dims[1] * k0)] = 1.0
    out = orc.filter27(dims, f).reshape(dims[2], dims[1], dims[0])
    # weights 1, 1/2, 1/4, 1/8 for self, face, edge and corner neighbours,
    # normalised to a sum of one
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                m = abs(di) + abs(dj) + abs(dk)
                want = [1.0, 0.5, 0.25, 0.125][m] / 8.0
                assert abs(out[k0 + dk, j0 + dj, i0 + di] - want) < 1e-15
    assert abs(out.sum() - 1.0) < 1e-14
    assert np.count_nonzero(out) == 27


def test_sum_is_kept_and_the_highest_mode_removed(orc):
    dims = (8, 6, 4)
    rng = np.random.default_rng(1)
    f = rng.standard_normal(3 * int(np.prod(dims)))
    g = orc.filter27(dims, f)
    n = int(np.prod(dims))
    for c in range(3):
        assert abs(g[c * n:(c + 1) * n].sum() - f[c * n:(c + 1) * n].sum()) < 1e-12
    i, j, k = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    cb = ((-1.0) ** (i + j + k)).transpose(2, 1, 0).reshape(-1)
    assert np.abs(orc.filter27(dims, cb)).max() < 1e-15
    # a smooth mode is damped by cos^2(k/2) per axis
    kx = 2 * np.pi / dims[0]
    wave = np.cos(kx * i).transpose(2, 1, 0).reshape(-1)
    assert np.allclose(orc.filter27(dims, wave), np.cos(kx / 2) ** 2 * wave, atol=1e-14)


def _div(dims, J):
    n = int(np.prod(dims))
    out = np.zeros(n)
    F = [J[c * n:(c + 1) * n].reshape(dims[2], dims[1], dims[0]) for c in range(3)]
    out = (F[0] - np.roll(F[0], 1, axis=2)) + (F[1] - np.roll(F[1], 1, axis=1)) + (F[2] - np.roll(F[2], 1, axis=0))
    return out.reshape(-1)


def test_commutes_with_the_discrete_divergence(orc):
    dims = (6, 5, 7)
    rng = np.random.default_rng(2)
    J = rng.standard_normal(3 * int(np.prod(dims)))
    assert np.allclose(_div(dims, orc.filter27(dims, J)), orc.filter27(dims, _div(dims, J)), atol=1e-13)


def test_gauss_law_with_smoothed_charge_over_a_run(orc):
    dims, ppc = (6, 6, 6), 6
    rng = np.random.default_rng(3)
    st = orc.State(dims, 0.5, 10.0, 2 * ppc, [(-1.0, 1.0), (1.0, 1.0)])
    st.filter = True
    npairs = ppc * int(np.prod(dims))
    x = rng.uniform(0, 6, (npairs, 3))
    st.add_particles(0, x, 0.3 * rng.standard_normal((npairs, 3)))
    st.add_particles(1, x, 0.3 * rng.standard_normal((npairs, 3)))
    st.step(30)
    d = st.diag()
    assert d["gauss_max"] < 1e-13, d["gauss_max"]
    # without the smoothing in the diagnostic the same fields break Gauss's law
    st.filter = False
    assert st.diag()["gauss_max"] > 1e-6
