"""ctypes binding of the FP64 CPU oracle (``pic_oracle.c``).

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It shares no code with
the GPU library: the two meet only through plain numpy arrays.

Every wrapper names the passage of Melzani et al. (arXiv:1308.5892) that the C
function follows; the C file states the readings taken where the paper is
silent or garbled.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


_LIB_NATIVE = os.path.join(_HERE, "liboracle_native.so")


def build(force: bool = True) -> str:
    """Compile liboracle.so next to its source with gcc (plain C11, -O2): the
    serial oracle that the tests and the smoke check use."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_native() -> str:
    """The same source built for timing the oracle on this host's cores:
    -O3 -march=native with OpenMP (parallel particle loops, one current array
    per thread added in thread order)."""
    tmp = _LIB_NATIVE + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-march=native", "-fopenmp", "-std=c11", "-fPIC", "-shared", "-o", tmp,
                           _SRC, "-lm"])
    os.replace(tmp, _LIB_NATIVE)
    return _LIB_NATIVE


_lib = None
_lib_native = None


def lib_native():
    """Handle of the native OpenMP build, compiled on its first use in the
    process (-march=native is this host's: a copy built elsewhere is never
    loaded)."""
    global _lib_native
    if _lib_native is None:
        build_native()
        _lib_native = _bind(C.CDLL(_LIB_NATIVE))
    return _lib_native


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _bind(C.CDLL(_LIB))
    return _lib


def _bind(L):
    """Argument types of every oracle entry point on a loaded build."""
    G = np.ctypeslib.ndpointer(dtype=np.int32, shape=(3,), flags="C_CONTIGUOUS")
    L.orc_curl_e.argtypes = [G, _dp, _dp]
    L.orc_curl_b.argtypes = [G, _dp, _dp]
    L.orc_advance_b.argtypes = [G, C.c_double, _dp, _dp]
    L.orc_advance_e.argtypes = [G, C.c_double, _dp, _dp]
    L.orc_gather.argtypes = [G, _dp, _dp, _dp, _dp, _dp]
    L.orc_boris.argtypes = [C.c_double, C.c_double, _dp, _dp, _dp]
    L.orc_deposit_move.argtypes = [G, C.c_double, _dp, _dp, _dp]
    L.orc_deposit_move.restype = C.c_int
    L.orc_deposit_charge.argtypes = [G, C.c_double, _dp, _dp]
    L.orc_step.argtypes = [G, C.c_double, C.c_double, C.c_int, _dp, _dp, C.c_int64,
                           _ip, _dp, _dp, _dp, _dp, C.c_int, C.c_int, C.c_int, C.c_int]
    L.orc_curl_e4.argtypes = [G, _dp, _dp]
    L.orc_advance_b4.argtypes = [G, C.c_double, _dp, _dp]
    L.orc_filter27.argtypes = [G, C.c_int, _dp]
    L.orc_wall_fields.argtypes = [G, C.c_int, _dp, _dp]
    L.orc_backward_half.argtypes = [G, C.c_double, _dp, C.c_int64, _ip, _dp, _dp, _dp, _dp]
    L.orc_diag.argtypes = [G, C.c_double, C.c_double, C.c_int, _dp, _dp, _dp, C.c_int64,
                           _ip, _dp, _dp, _dp, _dp, _dp, C.c_int, C.c_double, C.c_double,
                           C.c_void_p, C.c_int, C.c_int, C.c_int]
    L.orc_philox4x64.argtypes = [_up, _up, _up]
    L.orc_mj_range.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.orc_mj_table.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, _dp]
    L.orc_mj_radial.argtypes = [C.c_double, C.c_double]
    L.orc_mj_radial.restype = C.c_double
    L.orc_mj_draw.argtypes = [_dp, C.c_int, C.c_double, C.c_double, C.c_int, C.c_double,
                              C.c_double, C.c_double, _dp]
    L.orc_load_pairs.argtypes = [G, C.c_uint64, C.c_uint64, C.c_int64, C.c_int, C.c_int,
                                 C.c_double, C.c_double, C.c_double, _dp, _dp, C.c_int,
                                 C.c_double, C.c_double, C.c_int, C.c_double, C.c_double,
                                 C.c_int, _dp, _dp, _dp]
    L.orc_harris_params.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, _dp]
    L.orc_threads.argtypes = [C.c_int]
    L.orc_threads.restype = C.c_int
    return L


def _g(dims):
    return np.ascontiguousarray(dims, dtype=np.int32)


def _f(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------- fields

def curl_e(dims, e):
    """curl e at the b positions (App. A.3.2)."""
    out = np.zeros_like(_f(e))
    lib().orc_curl_e(_g(dims), _f(e), out)
    return out


def curl_e4(dims, e):
    """Fourth-order curl of e at the b positions (the fourth-order solver of
    App. A.3.2; reading in pic_oracle.c)."""
    out = np.zeros_like(_f(e))
    lib().orc_curl_e4(_g(dims), _f(e), out)
    return out


def advance_b4(dims, h, e, b):
    """Return b - h curl4 e (Faraday's law of the fourth-order solver)."""
    b = _f(b).copy()
    lib().orc_advance_b4(_g(dims), float(h), _f(e), b)
    return b


def curl_b(dims, b):
    """curl b at the e positions (App. A.3.2)."""
    out = np.zeros_like(_f(b))
    lib().orc_curl_b(_g(dims), _f(b), out)
    return out


def advance_b(dims, h, e, b):
    """Return b - h curl e (App. A.3.1 items 1 and 4 with h = dt/2)."""
    b = _f(b).copy()
    lib().orc_advance_b(_g(dims), float(h), _f(e), b)
    return b


def advance_e(dims, h, b, e):
    """Return e + h curl b (App. A.3.1 item 6 with h = dt)."""
    e = _f(e).copy()
    lib().orc_advance_e(_g(dims), float(h), _f(b), e)
    return e


def gather(dims, e, b, x):
    """Node-averaged, trilinearly weighted e and b at x (App. A.3.3)."""
    E = np.zeros(3)
    B = np.zeros(3)
    lib().orc_gather(_g(dims), _f(e), _f(b), _f(x), E, B)
    return E, B


def boris(k, h, E, B, u):
    """One relativistic Boris step of length h (App. A.3.3, eq. mover)."""
    u = _f(u).copy()
    lib().orc_boris(float(k), float(h), _f(E), _f(B), u)
    return u


def deposit_move(dims, sgn, x0, x1, J=None):
    """Charge-conserving deposit of the straight move x0 -> x1 (App. A.3.4)."""
    n = int(np.prod(dims))
    J = np.zeros(3 * n) if J is None else J
    npieces = lib().orc_deposit_move(_g(dims), float(sgn), _f(x0), _f(x1), J)
    return J, npieces


def wall_fields(dims, wall, e, b):
    """Conducting-wall condition (App. A.4) on the wall plane of axis `wall`."""
    e, b = _f(e).copy(), _f(b).copy()
    lib().orc_wall_fields(_g(dims), int(wall), e, b)
    return e, b


def filter27(dims, f):
    """The 27-point current smoothing of App. A.3.4 on each component grid."""
    f = _f(f).copy()
    n = int(np.prod(dims))
    lib().orc_filter27(_g(dims), len(f) // n, f)
    return f


def plane_power_spectrum(dims, f, normal):
    """Power spectrum of a field component in the planes normal to axis
    `normal`, summed over the planes (Sect. 3.2.2, method of measurement):
    the 2-D DFT over the two other axes (a1 < a2) of each plane, |.|^2, summed
    over planes.  f: one component grid, index i + n0 (j + n1 k).  Returns
    an array [m2, m1].  The DFT is numpy's FFT."""
    F = np.asarray(f, dtype=np.float64).reshape(dims[2], dims[1], dims[0])
    ax = {0: 2, 1: 1, 2: 0}                     # grid axis -> array axis
    a1, a2 = [a for a in range(3) if a != normal]
    G = np.transpose(F, (ax[normal], ax[a2], ax[a1]))
    return (np.abs(np.fft.fft2(G, axes=(1, 2))) ** 2).sum(axis=0)


def deposit_charge(dims, sgn, x, rho=None):
    """CIC node weights of a particle at x (App. A.3.3)."""
    rho = np.zeros(int(np.prod(dims))) if rho is None else rho
    lib().orc_deposit_charge(_g(dims), float(sgn), _f(x), rho)
    return rho


# ------------------------------------------------------------- simulation

class State:
    """Plain FP64 PIC state: x^t, u^{t-dt/2}, e^t, b^{t-dt/2} (App. A.3.1)."""

    def __init__(self, dims, dt, n_x, rho0, species, L=None):
        """species: list of (q_over_e, m_over_me).  L: the oracle build to run
        (default: the serial parity build)."""
        self.L = lib() if L is None else L
        self.dims = tuple(int(d) for d in dims)
        self.n = int(np.prod(self.dims))
        self.dt = float(dt)
        self.alpha0 = 2.0 / (n_x * n_x * rho0)  # App. A.2, eq. alpha
        self.q = np.array([s[0] for s in species], dtype=np.float64)
        self.m = np.array([s[1] for s in species], dtype=np.float64)
        self.kq = self.q / self.m                # (q_s/e)(m_e/m_s), App. A.2
        self.sgn = np.sign(self.q)
        self.e = np.zeros(3 * self.n)
        self.b = np.zeros(3 * self.n)
        self.x = np.zeros((0, 3))
        self.u = np.zeros((0, 3))
        self.species = np.zeros(0, dtype=np.int32)
        self.filter = False                      # smooth the current (App. A.3.4)
        self.wall = -1                           # axis with conducting walls (App. A.4), -1: none
        self.faraday4 = False                    # fourth-order curl in Faraday's law (App. A.3.2)

    def add_particles(self, s, x, u):
        self.x = np.concatenate([self.x, _f(x).reshape(-1, 3)])
        self.u = np.concatenate([self.u, _f(u).reshape(-1, 3)])
        self.species = np.concatenate(
            [self.species, np.full(len(_f(x).reshape(-1, 3)), s, dtype=np.int32)])

    def step(self, nsteps=1):
        x = np.ascontiguousarray(self.x).reshape(-1)
        u = np.ascontiguousarray(self.u).reshape(-1)
        self.L.orc_step(_g(self.dims), self.dt, self.alpha0, len(self.kq), self.kq, self.sgn,
                       len(self.species), np.ascontiguousarray(self.species), x, u,
                       self.e, self.b, int(nsteps), int(self.filter), int(self.wall), int(self.faraday4))
        self.x = x.reshape(-1, 3)
        self.u = u.reshape(-1, 3)

    def backward_half(self):
        """u^0 -> u^{-dt/2} and b^0 -> b^{-dt/2} (App. A.3.1, before the loop)."""
        u = np.ascontiguousarray(self.u).reshape(-1).copy()
        x = np.ascontiguousarray(self.x).reshape(-1)
        self.L.orc_backward_half(_g(self.dims), self.dt, self.kq, len(self.species),
                                np.ascontiguousarray(self.species), x, u, self.e, self.b)
        self.u = u.reshape(-1, 3)
        self.b = self._advance_b(-0.5 * self.dt, self.e, self.b)

    def _advance_b(self, h, e, b):
        return (advance_b4 if self.faraday4 else advance_b)(self.dims, h, e, b)

    def b_at_t(self):
        """b^t = b^{t-dt/2} - (dt/2) curl e^t (App. A.3.1 item 1)."""
        return self._advance_b(0.5 * self.dt, self.e, self.b)

    def diag(self, nbins=0, lo=-4.0, hi=3.0):
        nsp = len(self.kq)
        out = np.zeros(8 + 6 * nsp)
        hist = np.zeros(max(nsp * nbins, 1), dtype=np.int64)
        x = np.ascontiguousarray(self.x).reshape(-1)
        u = np.ascontiguousarray(self.u).reshape(-1)
        self.L.orc_diag(_g(self.dims), self.dt, self.alpha0, nsp, self.kq, self.sgn, self.m,
                       len(self.species), np.ascontiguousarray(self.species), x, u,
                       self.e, self.b, out, int(nbins), float(lo), float(hi),
                       hist.ctypes.data if nbins > 0 else None, int(self.filter), int(self.wall),
                       int(self.faraday4))
        d = {
            "W_E": out[0:3].copy(), "W_B": out[3:6].copy(),
            "gauss_max": out[6], "gauss_rms": out[7],
            "K": np.array([out[8 + 6 * s] for s in range(nsp)]),
            "P": np.array([out[9 + 6 * s: 12 + 6 * s] for s in range(nsp)]),
            "count": np.array([out[12 + 6 * s] for s in range(nsp)]),
            "sum_gm1": np.array([out[13 + 6 * s] for s in range(nsp)]),
        }
        if nbins > 0:
            d["hist"] = hist.reshape(nsp, nbins)
        return d


# ---------------------------------------------------------------- loading

def philox4x64(ctr, key):
    """Philox4x64-10 block (Salmon et al., SC'11)."""
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64(np.ascontiguousarray(ctr, dtype=np.uint64),
                         np.ascontiguousarray(key, dtype=np.uint64), out)
    return out


def mj_range(mu, beta0):
    lo, hi = C.c_double(), C.c_double()
    lib().orc_mj_range(float(mu), float(beta0), C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def mj_table(theta, gamma_beta, N=1 << 16, nint=1 << 16):
    """Inverse CDF table of the p_y marginal (App. D, eq. distr_y)."""
    beta0 = gamma_beta / np.sqrt(1.0 + gamma_beta * gamma_beta)
    y = np.zeros(N + 1)
    lib().orc_mj_table(1.0 / theta, beta0, int(N), int(nint), y)
    return y


def mj_radial(a, w):
    """r = sqrt(u^2-1) from l(x) = w l(a) (App. D, eq. finding_u)."""
    return lib().orc_mj_radial(float(a), float(w))


def load_pairs(dims, seed, stream, npairs, A, B, profile=0, paxis=0, centre=0.0, L=1.0,
               halfw=1.0, N=1 << 16, tabA=None, tabB=None, lib_=None):
    """Co-located pairs (Sect. 2.1) with drifting Maxwell-Juttner momenta (App. D).

    A, B: dicts with theta, gb (signed Gamma*beta) and axis (drift axis).
    Returns (x, uA, uB) as (npairs, 3) arrays.
    """
    tabA = mj_table(A["theta"], A["gb"], N) if tabA is None else tabA
    tabB = mj_table(B["theta"], B["gb"], N) if tabB is None else tabB
    x = np.zeros(3 * npairs)
    uA = np.zeros(3 * npairs)
    uB = np.zeros(3 * npairs)
    (lib() if lib_ is None else lib_).orc_load_pairs(_g(dims), int(seed), int(stream), int(npairs), int(profile),
                                                     int(paxis),
                         float(centre), float(L), float(halfw), _f(tabA), _f(tabB), int(N),
                         float(A["theta"]), float(A["gb"]), int(A["axis"]),
                         float(B["theta"]), float(B["gb"]), int(B["axis"]), x, uA, uB)
    return x.reshape(-1, 3), uA.reshape(-1, 3), uB.reshape(-1, 3)


def harris_params(theta_e, gu_e, chi=1.0, mi_over_me=1.0):
    """Relativistic Harris relations (App. C)."""
    out = np.zeros(6)
    lib().orc_harris_params(float(theta_e), float(gu_e), float(chi), float(mi_over_me), out)
    keys = ["wce_over_wpe_prime", "L_over_de_prime", "wce_over_wpe", "L_over_de",
            "theta_i", "gu_i"]
    return dict(zip(keys, out.tolist()))
