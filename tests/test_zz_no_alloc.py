"""pic_diag_noalloc (the diagnostics summed in the library's static device
scratch, for callers that cannot allocate) against pic_diag, through the C
ABI: two calls in a row, the second on a smaller box, in both forms; a box
beyond the scratch's size and unbinned particles are refused."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NB = 16


def _both(P, s, box, nsp):
    a, b = P.pic_diag_out(), P.pic_diag_out()
    ha = np.zeros(nsp * NB, dtype=np.int64)
    hb = np.full(nsp * NB, -7, dtype=np.int64)
    assert P.lib().pic_diag(s.ctx, box, C.byref(a), ha.ctypes.data) == P.PIC_OK
    assert P.lib().pic_diag_noalloc(s.ctx, box, C.byref(b), hb.ctypes.data) == P.PIC_OK
    return a, b, ha, hb


# charge density scale of the boxes below (alpha0 x particles per cell): the
# Gauss residual sits at FP64 roundoff of it, and the order of the FP64
# atomics that sum the charge moves it by a few ulp
RHO = 2.0 / (10.0 ** 2 * 8.0) * 8


def _same(a, b, ha, hb, nsp):
    # FP64 sums whose atomics may add in another order: equal to roundoff;
    # counts and histogram bins exactly
    def close(x, y):
        x, y = np.asarray(x, dtype=float), np.asarray(y, dtype=float)
        return np.all(np.abs(x - y) <= 1e-12 * np.maximum(np.abs(y), 1e-300) + 1e-300)
    assert close(a.W_E[:], b.W_E[:]) and close(a.W_B[:], b.W_B[:])
    assert close(a.K[:nsp], b.K[:nsp]) and close(a.sum_gm1[:nsp], b.sum_gm1[:nsp])
    for s in range(nsp):
        assert np.allclose(a.P[s][:], b.P[s][:], rtol=1e-12, atol=1e-9)
    assert abs(a.gauss_max - b.gauss_max) <= 1e-9 * a.gauss_max + 1e-13 * RHO
    assert abs(a.gauss_rms - b.gauss_rms) <= 1e-9 * a.gauss_rms + 1e-13 * RHO
    assert list(a.n_particles[:nsp]) == list(b.n_particles[:nsp])
    assert list(a.n_overflow[:nsp]) == list(b.n_overflow[:nsp])
    assert a.step == b.step and a.flags == b.flags == 0
    assert np.array_equal(ha, hb)


@pytest.mark.parametrize("fp64", [False, True])
def test_noalloc_diag_equals_pic_diag_on_two_calls(fp64):
    from paper_1308_5892_amd import pic as P
    big, small = (24, 20, 16), (8, 8, 8)
    boxes = [{"n": big, "n_x": 10.0, "rho0": 8.0, "max_particles": [4 * 24 * 20 * 16] * 2},
             {"n": small, "n_x": 10.0, "rho0": 8.0, "max_particles": [4 * 512] * 2}]
    s = P.Simulation(boxes, [(-1.0, 1.0), (1.0, 1.0)], 0.5, fp64=fp64, hist_bins=NB, hist_lo=-4.0, hist_hi=2.0)
    s.load(0, 0, 1, (0.3, 0.0, 1), (0.3, 0.0, 1), 4, seed=1)
    s.load(1, 0, 1, (0.05, 0.2, 0), (0.05, -0.2, 0), 4, seed=2)
    s.step(6)
    a, b, ha, hb = _both(P, s, 0, 2)          # the larger box first
    _same(a, b, ha, hb, 2)
    assert b.n_particles[0] == 4 * 24 * 20 * 16 and ha.sum() == 2 * 4 * 24 * 20 * 16
    a2, b2, ha2, hb2 = _both(P, s, 1, 2)      # then the smaller one: nothing of the first call remains
    _same(a2, b2, ha2, hb2, 2)
    assert b2.n_particles[0] == 4 * 512 and hb2.sum() == 2 * 4 * 512
    assert b2.gauss_max < 1e-4 * 2.0 / (100.0 * 8.0) * 4
    s.step(3)                                  # and again after more steps, the same context
    a3, b3, ha3, hb3 = _both(P, s, 1, 2)
    _same(a3, b3, ha3, hb3, 2)
    s.close()


def test_noalloc_diag_refuses_unbinned_particles_and_oversized_boxes():
    from paper_1308_5892_amd import pic as P
    s = P.Simulation([{"n": (8, 8, 8), "n_x": 10.0, "rho0": 4.0, "max_particles": [1024, 1024]}],
                     [(-1.0, 1.0), (1.0, 1.0)], 0.5)
    s.load(0, 0, 1, (0.1, 0.0, 1), (0.1, 0.0, 1), 2, seed=3)
    o = P.pic_diag_out()
    assert P.lib().pic_diag_noalloc(s.ctx, 0, C.byref(o), None) == P.PIC_ESTATE
    s.step(1)
    assert P.lib().pic_diag_noalloc(s.ctx, 0, C.byref(o), None) == P.PIC_OK
    assert list(o.n_particles[:2]) == [1024, 1024]
    s.close()
    # 256 x 256 x 65 cells: 8 bytes per cell alone exceed the 32 MiB scratch
    s = P.Simulation([{"n": (256, 256, 65), "n_x": 10.0, "rho0": 4.0, "max_particles": [0, 0]}],
                     [(-1.0, 1.0), (1.0, 1.0)], 0.5)
    s.step(1)
    assert P.lib().pic_diag_noalloc(s.ctx, 0, C.byref(o), None) == P.PIC_ENOMEM
    assert b"32 MiB" in P.lib().pic_last_error(s.ctx)
    assert P.lib().pic_diag(s.ctx, 0, C.byref(o), None) == P.PIC_OK   # pic_diag uses the arena
    s.close()
