"""Parity of the gfx950 HIP path (called through the C ABI) with the FP64 CPU
oracle, element by element on identical seeded inputs.

Tolerances: the FP64 form follows the oracle to accumulated roundoff (1e-11);
the FP32 form is held to the per-particle bound of 1e-5 relative momentum after
10 steps, and per-step quantities to what FP32 rounding of O(1) arithmetic
chains allows (a few ulp of 2^-24 times the number of operations).
"""
import numpy as np
import pytest

from tests import gpu_cases as G

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fp64,tol", [(False, 2e-5), (True, 1e-12)])
def test_vacuum_fields_match_oracle(fp64, tol):
    dims = (10, 12, 7)                       # ragged tiles on every axis
    e0, b0 = G.oblique_mode(dims, (1, 2, 1), 0.5)
    s = G.sim(dims, 10.0, 2.0, [1, 1], fp64=fp64)
    s.set_fields(0, e0, b0)
    st = G.oracle_state(dims, 10.0, 2.0)
    st.e, st.b = e0.copy(), b0.copy()
    s.step(25)
    st.step(25)
    e, b, j = s.fields(0)
    assert np.max(np.abs(e - st.e)) < tol
    assert np.max(np.abs(b - st.b)) < tol
    assert np.all(j == 0)
    s.close()


def _random_particles(rng, dims, n):
    x = rng.uniform(0, 1, (n, 3)) * np.array(dims)
    # a share of particles sit on or next to cell faces
    k = n // 8
    x[:k, 0] = np.floor(x[:k, 0]) + rng.choice([0.0, 1e-7, 1 - 1e-7], k)
    u = rng.standard_normal((n, 3)) * 0.5
    u[:k // 2] *= 8.0                         # relativistic tail, many crossings
    return x, u


@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("dims", [(9, 8, 6), (12, 12, 12), (4, 12, 12)])
def test_one_step_on_frozen_fields(fp64, dims):
    # ragged tiles; full 4x4x4 tiles, 3 per axis; one tile spanning x: the
    # re-binning takes its general and its full-tile form
    rng = np.random.default_rng(42)
    n = 3000
    s = G.sim(dims, 10.0, 40.0, [n, n], fp64=fp64)
    st = G.oracle_state(dims, 10.0, 40.0)
    e, b = G.random_fields(rng, int(np.prod(dims)), 0.05, 0.3)
    # both start from the state rounded to the library's storage format
    G.start(s, st, [_random_particles(rng, dims, n) for _ in range(2)], e=e, b=b, fp64=fp64)
    s.step(1)
    st.step(1)
    e1, b1, _ = s.fields(0)
    for sp in range(2):
        x, u, ids = s.particles(0, sp)
        assert np.array_equal(ids, np.arange(n))
        ref_u = st.u[st.species == sp]
        ref_x = st.x[st.species == sp]
        du = G.u_rel_err(u, ref_u, 1e-3)
        dx = np.abs(G.wrap_delta(x, ref_x, dims))
        if fp64:
            assert du.max() < 1e-12 and dx.max() < 1e-12
        else:
            assert du.max() < 2e-6, du.max()
            assert dx.max() < 2e-6, dx.max()
    tol = 1e-12 if fp64 else 2e-6
    assert np.max(np.abs(b1 - st.b)) < tol * np.abs(st.b).max()
    assert np.max(np.abs(e1 - st.e)) < tol * np.abs(st.e).max()
    s.close()


def test_deposit_alone_equals_oracle_current():
    # from e = b = 0 one step leaves e = alpha0 * sum sgn dV exactly: the
    # current of the split-segment deposit, compared face by face
    rng = np.random.default_rng(7)
    dims = (6, 7, 5)
    n = 4000
    for fp64 in (False, True):
        s = G.sim(dims, 10.0, 16.0, [n, n], fp64=fp64)
        st = G.oracle_state(dims, 10.0, 16.0)
        G.start(s, st, [_random_particles(rng, dims, n) for _ in range(2)], fp64=fp64)
        s.step(1)
        st.step(1)
        e1, _, _ = s.fields(0)
        scale = np.abs(st.e).max()
        err = np.max(np.abs(e1 - st.e)) / scale
        assert err < (1e-13 if fp64 else 1e-6), err
        s.close()


@pytest.mark.parametrize("fp64,tol", [(False, 1e-5), (True, 1e-11)])
def test_thermal_pair_plasma_ten_steps(fp64, tol):
    # 16^3 cells, 8 pairs per cell, theta = 0.1 (the small thermal workload):
    # per-particle momentum after 10 steps
    dims, ppc = (16, 16, 16), 8
    npairs = ppc * int(np.prod(dims))
    s = G.sim(dims, 10.0, 2 * ppc, [npairs, npairs], fp64=fp64)
    st = G.oracle_state(dims, 10.0, 2 * ppc)
    mj = {"theta": 0.1, "gb": 0.0, "axis": 1}
    parts = G.oracle_loaded(dims, 0.5, 10.0, 2 * ppc, G.PAIR,
                            [dict(seed=1, stream=0, npairs=npairs, A=mj, B=mj)])
    G.start(s, st, parts, fp64=fp64)
    s.step(10)
    st.step(10)
    worst = 0.0
    for sp in range(2):
        x, u, _ = s.particles(0, sp)
        ref = st.u[st.species == sp]
        worst = max(worst, G.u_rel_err(u, ref, 1e-2).max())
        assert np.abs(G.wrap_delta(x, st.x[st.species == sp], dims)).max() < 100 * tol
    assert worst < tol, worst
    d = s.diag(0)
    ref = st.diag()
    assert d["flags"] == 0
    rel = 1e-10 if fp64 else 1e-4
    assert abs(d["K"].sum() - ref["K"].sum()) < rel * ref["K"].sum()
    assert abs(d["W_E"].sum() - ref["W_E"].sum()) < rel * 10 * ref["W_E"].sum()
    s.close()


@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("case", ["rest", "beam_x", "harris"])
def test_loader_matches_oracle(fp64, case):
    from oracle import oracle as O
    dims = (24, 12, 4)
    if case == "rest":
        A = {"theta": 0.1, "gb": 0.0, "axis": 1}
        B = {"theta": 0.1, "gb": 0.0, "axis": 1}
        prof = dict(profile=0)
        ppc = 3
        npairs = ppc * int(np.prod(dims))
    elif case == "beam_x":
        A = {"theta": 0.01, "gb": np.sqrt(8.0), "axis": 0}
        B = {"theta": 0.01, "gb": -np.sqrt(8.0), "axis": 0}
        prof = dict(profile=0)
        ppc = 2
        npairs = ppc * int(np.prod(dims))
    else:
        A = {"theta": 1.0, "gb": -0.68, "axis": 2}
        B = {"theta": 0.04, "gb": 0.68, "axis": 2}
        prof = dict(profile=1, paxis=0, centre=6.0, L=3.5, halfw=6.0)
        ppc = 4
        npairs = int(round(ppc * (np.prod(dims) / dims[0]) * 2 * 3.5 * np.tanh(6.0 / 3.5)))
    s = G.sim(dims, 10.0, 2 * ppc, [npairs, npairs], fp64=fp64,
              species=[(-1.0, 1.0), (1.0, 1.0 if case != "harris" else 25.0)])
    kw = {}
    if case == "harris":
        kw = dict(profile=1, profile_axis=0, centre=6.0, thickness=3.5, half_width=6.0)
    s.load(0, 0, 1, (A["theta"], A["gb"], A["axis"]), (B["theta"], B["gb"], B["axis"]), ppc, seed=9,
           stream=4, **kw)
    x_ref, ua_ref, ub_ref = O.load_pairs(dims, 9, 4, npairs, A, B, **prof)
    for sp, uref in ((0, ua_ref), (1, ub_ref)):
        x, u, ids = s.particles(0, sp)
        assert len(x) == npairs
        assert np.array_equal(ids, np.arange(npairs))
        dx = np.abs(G.wrap_delta(x, x_ref, dims)).max()
        du = G.u_rel_err(u, uref, 1e-3).max()
        if fp64:
            assert dx < 1e-12 and du < 1e-9, (dx, du)
        else:
            assert dx < 2e-6 and du < 2e-7, (dx, du)
    s.close()


def test_gauss_law_and_determinism_fp32():
    dims, ppc = (12, 12, 12), 8
    npairs = ppc * int(np.prod(dims))
    runs = []
    for _ in range(2):
        s = G.sim(dims, 10.0, 2 * ppc, [npairs, npairs])
        s.load(0, 0, 1, (0.1, 0.0, 1), (0.1, 0.0, 1), ppc, seed=3)
        s.step(60)
        d = s.diag(0)
        e, b, _ = s.fields(0)
        runs.append((e, b, d))
        s.close()
    # int64 fixed-point currents make the fields independent of the order of the atomics
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])
    d = runs[0][2]
    rho_scale = 2.0 / (10.0 ** 2 * 2 * ppc) * ppc      # alpha0 times the pairs per cell
    assert d["gauss_max"] < 1e-4 * rho_scale, d["gauss_max"]


def test_runs_are_bitwise_identical_when_particles_overflow():
    # Which particles land in the overflow region (and take the HBM gather and
    # deposit instead of the tile's LDS ones) depends on the order of the slot
    # claims, which differs from run to run.  Both paths compute the same
    # arithmetic, so two runs still agree bit for bit: particles, e and b.
    def run():
        rng = np.random.default_rng(11)
        dims, n = (16, 8, 8), 6000
        s = G.sim(dims, 10.0, 16.0, [n, n], headroom=1.05)
        st = G.oracle_state(dims, 10.0, 16.0)
        parts = []
        for sp in range(2):
            x = rng.uniform(0, 1, (n, 3)) * np.array([4.0, 8.0, 8.0])
            u = 0.05 * rng.standard_normal((n, 3))
            u[: n // 10, 0] += 3.0
            parts.append((x, u))
        G.start(s, st, parts)
        seen = 0
        for _ in range(12):
            s.step(1)
            seen = max(seen, int(s.diag(0)["n_overflow"].sum()))
        out = [s.particles(0, sp) for sp in range(2)] + [s.fields(0)[:2]]
        s.close()
        return out, seen

    (a, seen), (b, _) = run(), run()
    assert seen > 0
    for sp in range(2):
        for k in range(3):
            assert np.array_equal(a[sp][k], b[sp][k]), (sp, k)
    assert np.array_equal(a[2][0], b[2][0]) and np.array_equal(a[2][1], b[2][1])


def test_long_magnetized_runs_are_bitwise_identical():
    # a hot electron-ion plasma in a uniform b for 2000 steps with repacks
    # every 50 steps: the whole state of two runs agrees bit for bit
    def run():
        n_x, ppc = 25, 8
        n = n_x ** 3
        s = G.sim((n_x,) * 3, float(n_x), 16.0, [ppc * n] * 2, dt=2 * np.pi * n_x / 1000,
                  species=[(-1.0, 1.0), (1.0, 49.0)], sort_interval=50)
        b = np.zeros(3 * n)
        b[2 * n:] = 1.0 / n_x
        s.set_fields(0, np.zeros(3 * n), b)
        s.load(0, 0, 1, (0.0016, 0.0, 2), (0.0016 / 49, 0.0, 2), ppc, seed=11)
        s.step(2000)
        out = [s.particles(0, sp) for sp in range(2)] + [s.fields(0)[:2]]
        s.close()
        return out

    a, b = run(), run()
    for sp in range(2):
        for k in range(3):
            assert np.array_equal(a[sp][k], b[sp][k]), (sp, k)
    assert np.array_equal(a[2][0], b[2][0]) and np.array_equal(a[2][1], b[2][1])


def test_gauss_law_fp64_at_roundoff():
    dims, ppc = (12, 10, 8), 6
    npairs = ppc * int(np.prod(dims))
    s = G.sim(dims, 10.0, 2 * ppc, [npairs, npairs], fp64=True)
    s.load(0, 0, 1, (0.3, 0.5, 0), (0.3, -0.5, 0), ppc, seed=5)
    s.step(40)
    d = s.diag(0)
    assert d["gauss_max"] < 1e-13, d["gauss_max"]
    s.close()


# FP32 bounds of the cases below, against the FP64 oracle: per-particle
# momentum 1e-5 relative (the bound of the ten-step thermal case), fields
# 1e-4 of their largest value when the plasma drives them (the current of
# ~1e3 moves per face rounded to FP32 once per step) and 2e-5 for fields
# given at the start (FP32 Yee arithmetic, as in the vacuum case)
U32, E32, F32 = 1e-5, 1e-4, 2e-5


@pytest.mark.parametrize("fp64", [False, True])
def test_overflow_region_keeps_parity(fp64):
    # all particles start in the first quarter of x and a tenth of them stream
    # to +x: the tiles they enter were laid out (almost) empty, so their
    # segments are full at once and the overflow region (HBM slow path) takes
    # the excess; the region holds 1024 particles per species here
    rng = np.random.default_rng(11)
    dims = (16, 8, 8)
    n = 6000
    s = G.sim(dims, 10.0, 16.0, [n, n], fp64=fp64, headroom=1.05)
    st = G.oracle_state(dims, 10.0, 16.0)
    parts = []
    for sp in range(2):
        x = rng.uniform(0, 1, (n, 3)) * np.array([4.0, 8.0, 8.0])
        u = 0.05 * rng.standard_normal((n, 3))
        u[: n // 10, 0] += 3.0
        parts.append((x, u))
    G.start(s, st, parts, fp64=fp64)
    seen = 0
    for _ in range(12):
        s.step(1)
        st.step(1)
        seen = max(seen, int(s.diag(0)["n_overflow"].sum()))
    assert seen > 0
    for sp in range(2):
        x, u, _ = s.particles(0, sp)
        assert len(x) == n
        assert G.u_rel_err(u, st.u[st.species == sp], 1e-3).max() < (1e-11 if fp64 else U32)
    e, _, _ = s.fields(0)
    assert np.max(np.abs(e - st.e)) < (1e-12 if fp64 else E32 * np.abs(st.e).max())
    s.close()


@pytest.mark.parametrize("fp64", [False, True])
def test_overflow_watch_repacks_early(fp64):
    # no periodic repack: an eighth of the particles stream into tiles laid
    # out empty, the overflow region (1024 particles per species) fills past
    # half, and the overflow watch, written by the e update into host memory,
    # has pic_step repack before the region runs out; nothing is lost and the
    # run follows the oracle
    from paper_1308_5892_amd import pic as P
    rng = np.random.default_rng(12)
    dims = (16, 8, 8)
    n = 6000
    s = G.sim(dims, 10.0, 16.0, [n, n], fp64=fp64, headroom=1.05, sort_interval=0)
    st = G.oracle_state(dims, 10.0, 16.0)
    parts = []
    for sp in range(2):
        x = rng.uniform(0, 1, (n, 3)) * np.array([4.0, 8.0, 8.0])
        u = 0.05 * rng.standard_normal((n, 3))
        u[: n // 8, 0] += 3.0
        parts.append((x, u))
    G.start(s, st, parts, fp64=fp64)
    P.pic_set_timing(s.ctx, 1)
    seen = 0
    for _ in range(20):
        s.step(1)
        st.step(1)
        seen = max(seen, int(s.diag(0)["n_overflow"].max()))
    assert seen > 512, seen                  # the watch limit: half the region
    assert P.pic_get_timing(s.ctx)["sort_launches"] >= 1
    assert s.diag(0)["flags"] == 0
    for sp in range(2):
        x, u, _ = s.particles(0, sp)
        assert len(x) == n
        assert G.u_rel_err(u, st.u[st.species == sp], 1e-3).max() < (1e-11 if fp64 else U32)
    s.close()


@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("dims,tile", [((1, 1, 1), (4, 4, 4)), ((3, 2, 5), (2, 1, 8)), ((7, 9, 2), (8, 2, 1))])
def test_tiny_and_odd_boxes(dims, tile, fp64):
    rng = np.random.default_rng(3)
    n = 200
    s = G.sim(dims, 10.0, 16.0, [n, n], fp64=fp64, tile=tile)
    st = G.oracle_state(dims, 10.0, 16.0)
    e, b = G.random_fields(rng, int(np.prod(dims)), 0.02, 0.2)
    G.start(s, st, [_random_particles(rng, dims, n) for _ in range(2)], e=e, b=b, fp64=fp64)
    s.step(5)
    st.step(5)
    for sp in range(2):
        x, u, _ = s.particles(0, sp)
        assert G.u_rel_err(u, st.u[st.species == sp], 1e-3).max() < (1e-11 if fp64 else U32)
    e1, b1, _ = s.fields(0)
    assert np.max(np.abs(e1 - st.e)) < (1e-12 if fp64 else F32 * np.abs(st.e).max())
    assert np.max(np.abs(b1 - st.b)) < (1e-12 if fp64 else F32 * np.abs(st.b).max())
    s.close()


@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("dims,tile", [((12, 8, 6), (8, 8, 4)), ((16, 12, 5), (8, 4, 4))])
def test_cell_codes_at_the_largest_tiles(dims, tile, fp64):
    # a binned particle keeps its cell as a one-byte code local to its tile;
    # 8x8x4 tiles use all 256 codes, and these boxes end in partial tiles
    # (x: 4 of 8 cells, z: 2 of 4; y: 4 of 4, z: 1 of 4), whose codes must
    # give the cells back through the hand-over, the repack and the read-back
    from paper_1308_5892_amd import pic as P
    rng = np.random.default_rng(43)
    n = 1500
    s = G.sim(dims, 10.0, 16.0, [n, n], fp64=fp64, tile=tile, sort_interval=3)
    st = G.oracle_state(dims, 10.0, 16.0)
    e, b = G.random_fields(rng, int(np.prod(dims)), 0.02, 0.2)
    G.start(s, st, [_random_particles(rng, dims, n) for _ in range(2)], e=e, b=b, fp64=fp64)
    P.pic_set_timing(s.ctx, 1)                    # counts the repacks
    s.step(7)
    st.step(7)
    assert P.pic_get_timing(s.ctx)["sort_launches"] >= 2
    for sp in range(2):
        x, u, _ = s.particles(0, sp)
        assert len(x) == n
        assert np.all((x >= 0) & (x < np.array(dims, float)))
        assert G.u_rel_err(u, st.u[st.species == sp], 1e-3).max() < (1e-11 if fp64 else U32)
    d = s.diag(0)
    assert d["flags"] == 0 and int(d["count"].sum()) == 2 * n
    s.close()


@pytest.mark.parametrize("fp64,tol", [(False, 1e-5), (True, 1e-11)])
@pytest.mark.parametrize("dims", [(2048, 2, 2), (2, 2048, 2), (2, 2, 1024)])
def test_largest_box_edges(dims, fp64, tol):
    # the largest edge the packed cell holds on each axis, with a quarter of
    # the particles in the last two cells along it, streaming through the
    # periodic boundary at the top index, and a quarter in the first two
    rng = np.random.default_rng(17)
    a = int(np.argmax(dims))
    n = 4 * int(np.prod(dims))
    tile = [2, 2, 2]
    tile[a] = 8
    s = G.sim(dims, 10.0, 8.0, [n, n], fp64=fp64, tile=tuple(tile))
    st = G.oracle_state(dims, 10.0, 8.0)
    parts = []
    for sp in range(2):
        x, u = _random_particles(rng, dims, n)
        q = n // 4
        x[:q, a] = dims[a] - 2.0 * rng.uniform(0, 1, q)
        u[:q, a] = np.abs(u[:q, a]) + 0.5
        x[q:2 * q, a] = 2.0 * rng.uniform(0, 1, q)
        u[q:2 * q, a] = -np.abs(u[q:2 * q, a]) - 0.5
        parts.append((x, u))
    G.start(s, st, parts, fp64=fp64)
    s.step(10)
    st.step(10)
    for sp in range(2):
        x, u, _ = s.particles(0, sp)
        assert len(x) == n
        assert G.u_rel_err(u, st.u[st.species == sp], 1e-2).max() < tol
        assert np.abs(G.wrap_delta(x, st.x[st.species == sp], dims)).max() < 100 * tol
        assert np.all((x >= 0) & (x < np.array(dims)))
    e1, _, _ = s.fields(0)
    assert np.max(np.abs(e1 - st.e)) < (1e-11 if fp64 else 1e-4) * np.abs(st.e).max()
    d = s.diag(0)
    assert d["flags"] == 0
    s.close()


@pytest.mark.parametrize("fp64,tol", [(False, 1e-5), (True, 1e-11)])
@pytest.mark.parametrize("species", [[(-1.0, 1.0)], [(-1.0, 1.0), (1.0, 1.0), (1.0, 25.0), (-1.0, 4.0)]],
                         ids=["one_species", "four_species"])
def test_one_and_four_species(species, fp64, tol):
    # the fewest and the most species a context takes, each with its own
    # random particles (not co-located, so the fields build up), 10 steps;
    # momenta, fields and the per-species diagnostics with a gamma-1
    # histogram against the oracle
    from paper_1308_5892_amd import pic as P
    rng = np.random.default_rng(29)
    dims, n, nbins = (10, 9, 8), 700, 24
    s = P.Simulation([{"n": dims, "n_x": 10.0, "rho0": 8.0, "max_particles": [n] * len(species)}], species, 0.5,
                     fp64=fp64, track_ids=True, hist_bins=nbins, hist_lo=-4.0, hist_hi=2.0)
    st = G.oracle_state(dims, 10.0, 8.0, species=species)
    G.start(s, st, [_random_particles(rng, dims, n) for _ in species], fp64=fp64)
    s.step(10)
    st.step(10)
    for sp in range(len(species)):
        x, u, _ = s.particles(0, sp)
        assert G.u_rel_err(u, st.u[st.species == sp], 1e-2).max() < tol, sp
        assert np.abs(G.wrap_delta(x, st.x[st.species == sp], dims)).max() < 100 * tol
    e, b, _ = s.fields(0)
    assert np.abs(e - st.e).max() < (1e-11 if fp64 else 1e-4) * np.abs(st.e).max()
    d, r = s.diag(0, hist_bins=nbins), st.diag(nbins, -4.0, 2.0)
    assert d["flags"] == 0
    assert np.allclose(d["K"], r["K"], rtol=1e-10 if fp64 else 1e-5)
    assert np.allclose(d["P"], r["P"], rtol=0, atol=(1e-10 if fp64 else 1e-5) * n)   # |u| ~ 1 per particle
    assert d["count"].tolist() == [n] * len(species)
    # histogram bins agree up to particles that sit on a bin edge within roundoff
    assert np.abs(d["hist"] - r["hist"]).sum() <= (0 if fp64 else 4), (d["hist"], r["hist"])
    s.close()


@pytest.mark.parametrize("fp64", [False, True])
def test_nonfinite_momentum_is_flagged_and_contained(fp64):
    # a NaN and an oversized momentum given from the host: the push flags
    # them (PIC_FLAG_NONFINITE, reported once as PIC_EFLAG by pic_diag), puts
    # those two particles at rest and goes on; every momentum stays finite
    # and no particle is lost
    import ctypes as C
    from paper_1308_5892_amd import pic as P
    rng = np.random.default_rng(31)
    dims, n = (8, 8, 8), 512
    s = G.sim(dims, 10.0, 8.0, [n, n], fp64=fp64)
    st = G.oracle_state(dims, 10.0, 8.0)           # only to share the storage rounding of the start
    parts = [_random_particles(rng, dims, n) for _ in range(2)]
    G.start(s, st, parts, fp64=fp64)
    x0, u0 = G.to_storage(parts[0][0], parts[0][1], dims, fp64)
    bad = u0.copy()
    bad[5] = [np.nan, 0.0, 0.0]
    bad[7] = [1e20, 0.0, 0.0]
    s.set_particles(0, 0, x0, bad, np.arange(n))
    s.step(1)
    out = P.pic_diag_out()
    assert P.lib().pic_diag(s.ctx, 0, C.byref(out), None) == P.PIC_EFLAG
    assert out.flags & P.PIC_FLAG_NONFINITE
    assert P.lib().pic_diag(s.ctx, 0, C.byref(out), None) == P.PIC_OK     # reported once
    _, u, _ = s.particles(0, 0)
    assert np.all(np.isfinite(u)) and np.abs(u[[5, 7]]).max() < 1e-3
    assert s.diag(0)["count"].tolist() == [n, n]
    s.close()


def test_empty_plasma_and_zero_steps():
    s = G.sim((8, 8, 8), 10.0, 2.0, [0, 0])
    s.step(0)
    s.step(3)
    d = s.diag(0)
    assert d["count"].tolist() == [0, 0]
    assert d["W_E"].sum() == 0 and d["gauss_max"] == 0
    s.close()


@pytest.mark.parametrize("fp64", [False, True])
def test_repack_keeps_parity(fp64):
    dims, ppc = (12, 8, 8), 4
    npairs = ppc * int(np.prod(dims))
    s = G.sim(dims, 10.0, 2 * ppc, [npairs, npairs], fp64=fp64, sort_interval=3)
    st = G.oracle_state(dims, 10.0, 2 * ppc)
    parts = G.oracle_loaded(dims, 0.5, 10.0, 2 * ppc, G.PAIR,
                            [dict(seed=8, stream=0, npairs=npairs, A={"theta": 0.2, "gb": 0.3, "axis": 0},
                                  B={"theta": 0.2, "gb": -0.3, "axis": 0})])
    G.start(s, st, parts, fp64=fp64)
    from paper_1308_5892_amd import pic as P
    P.pic_set_timing(s.ctx, 1)
    s.step(10)
    st.step(10)
    assert P.pic_get_timing(s.ctx)["sort_launches"] >= 3
    for sp in range(2):
        _, u, _ = s.particles(0, sp)
        assert G.u_rel_err(u, st.u[st.species == sp], 1e-3).max() < (1e-11 if fp64 else U32)
    # timing mode 2 times the push launches only; other modes are refused
    P.pic_set_timing(s.ctx, 2)
    s.step(4)
    t = P.pic_get_timing(s.ctx)
    assert t["push_launches"] == 4 and t["push_ms"] > 0.0
    assert t["field_launches"] == 0 and t["sort_launches"] == 0
    with pytest.raises(P.PicError):
        P.pic_set_timing(s.ctx, 3)
    s.close()


def test_harris_field_and_backward_half_step():
    from oracle import oracle as O
    dims = (32, 8, 4)
    L, b0 = 3.0, 0.12
    npairs = 2000
    s = G.sim(dims, 15.0, 8.0, [npairs, npairs], fp64=True, species=[(-1.0, 1.0), (1.0, 25.0)])
    s.harris_field(0, 0, 1, b0, L, [8.0, 24.0])
    s.load(0, 0, 1, (1.0, -0.68, 2), (0.04, 0.68, 2), 4.0, seed=2, profile=1, profile_axis=0,
           centre=8.0, thickness=L, half_width=8.0)
    _, b, _ = s.fields(0)
    n = int(np.prod(dims))
    i = np.arange(n) % dims[0]
    ref = b0 * (np.tanh((i + 0.5 - 8.0) / L) - np.tanh((i + 0.5 - 24.0) / L) - 1.0)
    assert np.max(np.abs(b[n:2 * n] - ref)) < 1e-15          # e = 0: b^{-dt/2} = b^0
    assert np.all(b[:n] == 0) and np.all(b[2 * n:] == 0)
    # binned momenta are the loaded ones pushed back by dt/2 in b^0
    npairs_h = int(round(4.0 * (n / dims[0]) * 2 * L * np.tanh(8.0 / L)))
    A = {"theta": 1.0, "gb": -0.68, "axis": 2}
    B = {"theta": 0.04, "gb": 0.68, "axis": 2}
    x0, ua, ub = O.load_pairs(dims, 2, 0, npairs_h, A, B, profile=1, paxis=0, centre=8.0, L=L, halfw=8.0)
    st = O.State(dims, 0.5, 15.0, 8.0, [(-1.0, 1.0), (1.0, 25.0)])
    st.b[n:2 * n] = ref
    st.add_particles(0, x0, ua)
    st.add_particles(1, x0, ub)
    st.backward_half()
    for sp in range(2):
        _, u, _ = s.particles(0, sp)
        assert G.u_rel_err(u, st.u[st.species == sp], 1e-3).max() < 1e-10
    s.close()


@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("walls", [(0, 0, 0), (0, 2, 3)], ids=["periodic", "mixed_walls"])
def test_multiple_boxes_in_one_launch(walls, fp64):
    # three boxes of different shapes in one launch; in the second case the
    # middle box has walls across y and the last across z, next to a
    # periodic box, so one launch runs both kinds of box
    from paper_1308_5892_amd import pic as P
    from oracle import oracle as O
    rng = np.random.default_rng(21)
    dims_list = [(8, 8, 8), (13, 6, 5), (4, 4, 12)]
    boxes, n = [], 500
    for d, w in zip(dims_list, walls):
        boxes.append({"n": d, "n_x": 10.0, "rho0": 8.0, "max_particles": [n, n], "walls": w})
    sim = P.Simulation(boxes, G.PAIR, 0.5, fp64=fp64, track_ids=True)
    states = []
    for bi, d in enumerate(dims_list):
        e, b = G.random_fields(rng, int(np.prod(d)), 0.02, 0.2)
        st = O.State(d, 0.5, 10.0, 8.0, G.PAIR)
        st.wall = walls[bi] - 1
        if st.wall >= 0:
            e, b = O.wall_fields(d, st.wall, e, b)   # start from fields that meet the walls' condition
        G.start(sim, st, [_random_particles(rng, d, n) for _ in range(2)], box=bi, e=e, b=b, fp64=fp64)
        states.append(st)
    sim.step(4)
    for bi, st in enumerate(states):
        st.step(4)
        for sp in range(2):
            _, u, _ = sim.particles(bi, sp)
            assert G.u_rel_err(u, st.u[st.species == sp], 1e-3).max() < (1e-11 if fp64 else U32)
        e, _, _ = sim.fields(bi)
        assert np.max(np.abs(e - st.e)) < (1e-12 if fp64 else E32 * np.abs(st.e).max())
    sim.close()


def test_load_beyond_capacity_after_binning_is_refused():
    # the capacity counts particles already binned by earlier loads and steps,
    # not only the staged ones: a second full load into a filled species is
    # refused with PIC_ENOMEM, and the context keeps running unharmed
    import ctypes as C
    from paper_1308_5892_amd import pic as P
    dims, ppc = (8, 8, 8), 2
    npairs = ppc * int(np.prod(dims))
    s = G.sim(dims, 10.0, 2 * ppc, [npairs, npairs])
    s.load(0, 0, 1, (0.1, 0.0, 1), (0.1, 0.0, 1), ppc, seed=1)
    s.step(2)
    d = P.load_desc(0, 0, 1, (0.1, 0.0, 1), (0.1, 0.0, 1), ppc, seed=2)
    assert P.lib().pic_load_maxwell_juttner(s.ctx, C.byref(d)) == P.PIC_ENOMEM
    # a load that fits next to the binned particles is still accepted (none here: full)
    d0 = P.load_desc(0, 0, 1, (0.1, 0.0, 1), (0.1, 0.0, 1), 0.0, seed=3)
    assert P.lib().pic_load_maxwell_juttner(s.ctx, C.byref(d0)) == P.PIC_OK
    s.step(3)
    out = s.diag(0)
    assert out["flags"] == 0 and out["count"].tolist() == [npairs, npairs]
    s.close()
    # half the capacity loaded twice fits
    s = G.sim(dims, 10.0, 2 * ppc, [2 * npairs, 2 * npairs])
    s.load(0, 0, 1, (0.1, 0.0, 1), (0.1, 0.0, 1), ppc, seed=1)
    s.step(1)
    s.load(0, 0, 1, (0.1, 0.0, 1), (0.1, 0.0, 1), ppc, seed=2)
    s.step(1)
    assert s.diag(0)["count"].tolist() == [2 * npairs, 2 * npairs]
    assert P.lib().pic_load_maxwell_juttner(s.ctx, C.byref(d)) == P.PIC_ENOMEM
    s.close()


def test_fp64_tiles_needing_more_lds_in_one_process():
    # FP64 contexts with 8x4x4 tiles (about 95 KB of LDS per block) and then
    # 8x8x4 tiles (about 162 KB): the second needs the kernel's LDS limit
    # raised again; both run and follow the oracle
    rng = np.random.default_rng(41)
    dims, n = (16, 8, 8), 800
    for tile in ((8, 4, 4), (8, 8, 4)):
        s = G.sim(dims, 10.0, 8.0, [n, n], fp64=True, tile=tile)
        st = G.oracle_state(dims, 10.0, 8.0)
        e, b = G.random_fields(rng, int(np.prod(dims)), 0.02, 0.2)
        G.start(s, st, [_random_particles(rng, dims, n) for _ in range(2)], e=e, b=b, fp64=True)
        s.step(3)
        st.step(3)
        for sp in range(2):
            _, u, _ = s.particles(0, sp)
            assert G.u_rel_err(u, st.u[st.species == sp], 1e-3).max() < 1e-11, tile
        assert s.diag(0)["flags"] == 0
        s.close()


# ------------------------------------------ fourth-order solver (PIC_FARADAY4)

@pytest.mark.parametrize("fp64,tol", [(False, 2e-5), (True, 1e-12)])
def test_fourth_order_solver_vacuum_fields_match_oracle(fp64, tol):
    # random e and b (every wave number) in vacuum, 20 steps: the fourth-order
    # Faraday curl and Yee's Ampere curl against the oracle's
    rng = np.random.default_rng(51)
    dims = (10, 12, 7)
    n = int(np.prod(dims))
    e0, b0 = G.random_fields(rng, n, 0.3, 0.3)
    s = G.sim(dims, 10.0, 2.0, [1, 1], fp64=fp64, faraday4=True)
    st = G.oracle_state(dims, 10.0, 2.0)
    st.faraday4 = True
    G.start(s, st, [], e=e0, b=b0, fp64=fp64)
    s.step(20)
    st.step(20)
    e, b, _ = s.fields(0)
    assert np.max(np.abs(e - st.e)) < tol * np.abs(st.e).max()
    assert np.max(np.abs(b - st.b)) < tol * np.abs(st.b).max()
    s.close()


@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("dims", [(9, 8, 6), (12, 12, 12)])
def test_fourth_order_solver_one_step_on_frozen_fields(fp64, dims):
    # random particles in random fields: the gather at x^t uses b^t formed
    # with the fourth-order curl (in the tile and on the HBM path)
    rng = np.random.default_rng(43)
    n = 3000
    s = G.sim(dims, 10.0, 40.0, [n, n], fp64=fp64, faraday4=True)
    st = G.oracle_state(dims, 10.0, 40.0)
    st.faraday4 = True
    e, b = G.random_fields(rng, int(np.prod(dims)), 0.05, 0.3)
    G.start(s, st, [_random_particles(rng, dims, n) for _ in range(2)], e=e, b=b, fp64=fp64)
    s.step(1)
    st.step(1)
    tol = 1e-12 if fp64 else 2e-6
    for sp in range(2):
        x, u, _ = s.particles(0, sp)
        assert G.u_rel_err(u, st.u[st.species == sp], 1e-3).max() < tol
        assert np.abs(G.wrap_delta(x, st.x[st.species == sp], dims)).max() < tol
    e1, b1, _ = s.fields(0)
    assert np.max(np.abs(b1 - st.b)) < tol * np.abs(st.b).max()
    assert np.max(np.abs(e1 - st.e)) < tol * np.abs(st.e).max()
    s.close()


@pytest.mark.parametrize("fp64,tol", [(False, 1e-5), (True, 1e-11)])
def test_fourth_order_solver_thermal_ten_steps(fp64, tol):
    # a hot pair plasma (theta = 0.3) for 10 steps: per-particle momenta,
    # fields and the FP64 Gauss residual
    dims, ppc = (12, 10, 8), 6
    npairs = ppc * int(np.prod(dims))
    s = G.sim(dims, 10.0, 2 * ppc, [npairs, npairs], fp64=fp64, faraday4=True)
    st = G.oracle_state(dims, 10.0, 2 * ppc)
    st.faraday4 = True
    mj = {"theta": 0.3, "gb": 0.0, "axis": 1}
    parts = G.oracle_loaded(dims, 0.5, 10.0, 2 * ppc, G.PAIR, [dict(seed=7, stream=0, npairs=npairs, A=mj, B=mj)])
    G.start(s, st, parts, fp64=fp64)
    s.step(10)
    st.step(10)
    for sp in range(2):
        _, u, _ = s.particles(0, sp)
        assert G.u_rel_err(u, st.u[st.species == sp], 1e-2).max() < tol
    e, b, _ = s.fields(0)
    assert np.max(np.abs(e - st.e)) < (1e-11 if fp64 else 1e-4) * np.abs(st.e).max()
    d = s.diag(0)
    assert d["flags"] == 0
    if fp64:
        assert d["gauss_max"] < 1e-13
    s.close()
