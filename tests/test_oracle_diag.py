"""Pins of the oracle's diagnostics (orc_diag) against the exact motion in a
uniform field and against energy conservation with two masses.

* Kinetic energy K_s = sum (m_s/m_e)(gamma^t - 1) and momentum P_s = sum u^t,
  both at the diagnostic time t (App. A.2 normalisation; Sect. 3.1 uses the
  k = 0 momentum sum for F(omega); Sect. 3.1.3 the energy curves): in a
  uniform e with b = 0 the mover's kicks are exact, so after n steps the
  momentum at time t = n dt is u0 + k e t and gamma^t = sqrt(1 + |u0 + k e t|^2)
  - the solution of du/dt = k e, not a restatement of the diagnostic.
* The mass weight of K: a cold electron-ion k = 0 oscillation started from a
  uniform e converts the field energy into kinetic energy shared as
  m_i : m_e inversely (equal and opposite momenta), and the total stays
  constant only when the heavy species is weighted by its mass.
* The log10(gamma - 1) histogram: hand-placed gammas in known bins, both end
  bins reached by clamping, and gamma = 1 (log of zero) in the lowest bin.
"""
import numpy as np


def _tiny_coupling_state(orc, dims, species, dt=0.5):
    # rho0 so large that alpha0 ~ 1e-16: the particles' current leaves e
    # unchanged to roundoff, so the fields are external
    return orc.State(dims, dt, n_x=1.0, rho0=2e16, species=species)


def test_momentum_and_kinetic_energy_follow_the_exact_motion(orc):
    dims = (4, 3, 5)
    n = 4 * 3 * 5
    masses = [1.0, 4.0, 25.0]
    charges = [-1.0, 1.0, 2.0]
    st = _tiny_coupling_state(orc, dims, list(zip(charges, masses)))
    E0 = np.array([0.02, -0.035, 0.011])
    st.e[:] = np.repeat(E0, n)
    rng = np.random.default_rng(11)
    u0 = {}
    for s in range(3):
        x = rng.uniform(0, 1, (7, 3)) * np.array(dims)
        u = rng.normal(scale=0.6, size=(7, 3))
        u0[s] = u.copy()
        st.add_particles(s, x, u)
    st.backward_half()                    # u^{-dt/2} from u(0)
    for nstep in (0, 1, 6, 25):
        if nstep:
            st.step(nstep - st_steps)
        st_steps = nstep
        d = st.diag()
        t = nstep * st.dt
        for s in range(3):
            k = charges[s] / masses[s]
            ut = u0[s] + k * E0 * t           # exact momentum at time t
            gam = np.sqrt(1.0 + (ut ** 2).sum(1))
            assert np.allclose(d["P"][s], ut.sum(0), rtol=0, atol=1e-12), (nstep, s)
            assert abs(d["K"][s] - masses[s] * (gam - 1.0).sum()) < 1e-11 * max(1.0, masses[s] * gam.sum())
            assert abs(d["sum_gm1"][s] - (gam - 1.0).sum()) < 1e-11 * gam.sum()
            assert d["count"][s] == 7
    # the half-step offset a diagnostic on u^{t-dt/2} would carry is far above
    # the tolerance used: |k e dt/2| * 7 particles
    assert 7 * 0.5 * st.dt * 0.011 / 25 > 1e-6


def test_kinetic_energy_weights_the_heavy_species_by_its_mass(orc):
    # cold electrons and ions (m_i/m_e = 25) co-located on a lattice, at rest,
    # in a uniform e_x: a k = 0 oscillation.  Field energy turns into kinetic
    # energy with equal and opposite momenta, so the ions carry
    # m_e/(m_e + m_i) = 1/26 of it; total energy is conserved by the
    # leap-frog to O((w dt)^2).
    dims, n_x, dt, mi = (2, 2, 2), 10.0, 0.1, 25.0
    st = orc.State(dims, dt, n_x=n_x, rho0=2, species=[(-1, 1), (1, mi)])
    i, j, k = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    x = np.stack([i.ravel(), j.ravel(), k.ravel()], 1) + np.array([0.3, 0.6, 0.45])
    st.add_particles(0, x, np.zeros_like(x))
    st.add_particles(1, x, np.zeros_like(x))
    n = st.n
    st.e[:n] = 2e-3                       # uniform e_x, no charge needed
    st.backward_half()
    tot, share = [], []
    # quarter period of w_P = sqrt(1 + 1/25)/n_x: about 15.4 plasma units
    for _ in range(200):
        d = st.diag()
        W = d["W_E"].sum() + d["W_B"].sum()
        K = d["K"]
        tot.append(W + K.sum())
        if K.sum() > 0.5 * tot[0]:
            share.append(K[1] / K.sum())
        st.step(1)
    tot = np.array(tot)
    assert np.abs(tot / tot[0] - 1).max() < 1e-3
    # an unweighted ion term would lose ~96 % of the ions' share (~3.7 % of the total)
    assert len(share) > 20
    assert np.allclose(share, 1.0 / 26.0, rtol=2e-3, atol=0)


def test_gamma_histogram_bins_and_clamps(orc):
    # bins of log10(gamma - 1) over [lo, hi) = [-4, 3) in 7 bins of width 1
    nbins, lo, hi = 7, -4.0, 3.0
    # one particle per listed log10(gamma - 1); gamma - 1 = 0 is listed as None
    logs = [-3.5, -2.5, -2.5, -0.5, 0.25, 2.9, -7.0, 5.0, None, -1.0, 2.0, 3.4, -4.5]
    # bin of each, by hand: floor(v - lo) clamped to [0, 6]; -1.0 and 2.0 sit
    # on a bin's lower edge; 3.4 and -4.5 are one bin past either end (index 7
    # and -1 before the clamp)
    expect_bins = [0, 1, 1, 3, 4, 6, 0, 6, 0, 3, 6, 6, 0]
    gm1 = np.array([0.0 if v is None else 10.0 ** v for v in logs])
    # |u| from gamma; exact bin edges are kept off by choosing u slightly above
    gam = 1.0 + gm1
    u = np.sqrt(np.maximum(gam * gam - 1.0, 0.0))
    u[9] *= 1 + 1e-9
    u[10] *= 1 + 1e-9
    dims = (2, 2, 2)
    st = _tiny_coupling_state(orc, dims, [(-1, 1)])
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 2, (len(u), 3))
    direc = rng.normal(size=(len(u), 3))
    direc /= np.linalg.norm(direc, axis=1)[:, None]
    st.add_particles(0, x, u[:, None] * direc)
    d = st.diag(nbins=nbins, lo=lo, hi=hi)
    want = np.bincount(expect_bins, minlength=nbins)
    assert d["hist"].shape == (1, nbins)
    assert d["hist"][0].tolist() == want.tolist()
    assert want.tolist() == [4, 2, 0, 2, 1, 0, 4]
