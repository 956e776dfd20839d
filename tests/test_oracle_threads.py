"""The oracle's OpenMP build (-O3 -march=native -fopenmp, used only to time
the oracle on all host cores) against the serial parity build: the loader
draws the same particles (counter-based Philox per pair), and a few steps of
the cycle agree to roundoff - the per-thread currents are added in another
order than the serial sum, nothing else differs."""
import numpy as np


def test_openmp_build_equals_the_serial_oracle(orc):
    N = orc.lib_native()
    assert N.orc_threads(4) == 4
    dims, ppc, dt = (10, 9, 8), 6, 0.5
    npairs = ppc * int(np.prod(dims))
    sp = {"theta": 0.3, "gb": 0.2, "axis": 0}
    xs, uas, ubs = orc.load_pairs(dims, 5, 1, npairs, sp, sp)
    xn, uan, ubn = orc.load_pairs(dims, 5, 1, npairs, sp, sp, lib_=N)
    assert np.array_equal(xs, xn) and np.array_equal(uas, uan) and np.array_equal(ubs, ubn)
    states = []
    for L in (None, N):
        st = orc.State(dims, dt, 10.0, 2 * ppc, [(-1.0, 1.0), (1.0, 25.0)], L=L)
        st.add_particles(0, xs, uas)
        st.add_particles(1, xs, ubs)
        st.backward_half()
        st.step(8)
        states.append(st)
    s, n = states
    assert np.abs(s.u - n.u).max() < 1e-12
    assert np.abs(s.x - n.x).max() < 1e-12
    assert np.abs(s.e - n.e).max() < 1e-12 * np.abs(s.e).max()
    assert np.abs(s.b - n.b).max() < 1e-12 * np.abs(s.b).max()
    assert n.diag()["gauss_max"] < 1e-12 * s.alpha0 * ppc
    N.orc_threads(1)
