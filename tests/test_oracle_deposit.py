"""Pins of the oracle's charge-conserving current deposit (App. A.1, A.3.4).

The attributed volume change of eq. current_dep equals the charge swept by the
moving unit cube through each grid-B face: the test integrates, by Gauss-Legendre
quadrature along the straight path, the overlap area of the cube's cross-section
with every face (brute force, no use of the formula), for moves inside a cell and
for moves that cross one, two or three node planes.
"""
import numpy as np
import pytest

GL_X, GL_W = np.polynomial.legendre.leggauss(6)


def _ov(c, j):
    """overlap length of [c-1/2, c+1/2] with [j-1/2, j+1/2]"""
    return max(0.0, min(c + 0.5, j + 0.5) - max(c - 0.5, j - 0.5))


def _kinks(x0, x1):
    lam = [0.0, 1.0]
    for a in range(3):
        lo, hi = sorted((x0[a], x1[a]))
        for m in range(int(np.floor(lo)) - 1, int(np.ceil(hi)) + 2):
            if x1[a] != x0[a]:
                t = (m - x0[a]) / (x1[a] - x0[a])
                if 0 < t < 1:
                    lam.append(t)
    return sorted(lam)


def _swept_flux(x0, x1, a, node):
    """charge volume crossing the face normal to a at node[a]+1/2 (towards +a)"""
    b1, b2 = (a + 1) % 3, (a + 2) % 3
    D = np.asarray(x1) - np.asarray(x0)
    lam = _kinks(x0, x1)
    tot = 0.0
    for l0, l1 in zip(lam[:-1], lam[1:]):
        for xg, wg in zip(GL_X, GL_W):
            s = 0.5 * (l0 + l1) + 0.5 * (l1 - l0) * xg
            p = np.asarray(x0) + s * D
            plane = node[a] + 0.5
            if abs(p[a] - plane) < 0.5:
                tot += 0.5 * (l1 - l0) * wg * D[a] * _ov(p[b1], node[b1]) * _ov(p[b2], node[b2])
    return tot


def _check_move(orc, dims, x0, x1, sgn=1.0):
    J, npieces = orc.deposit_move(dims, sgn, x0, x1)
    n = int(np.prod(dims))
    lo = np.floor(np.minimum(x0, x1)).astype(int) - 1
    hi = np.floor(np.maximum(x0, x1)).astype(int) + 2
    seen = 0.0
    for a in range(3):
        for i in range(lo[0], hi[0] + 1):
            for j in range(lo[1], hi[1] + 1):
                for k in range(lo[2], hi[2] + 1):
                    node = (i, j, k)
                    ref = -sgn * _swept_flux(x0, x1, a, node)
                    idx = a * n + (i % dims[0]) + dims[0] * ((j % dims[1]) + dims[1] * (k % dims[2]))
                    got = J[idx]
                    assert abs(got - ref) < 1e-14, (a, node, got, ref)
                    seen += abs(got)
    # nothing outside the checked window
    assert abs(np.abs(J).sum() - seen) < 1e-13
    return npieces


def test_deposit_within_cell_matches_swept_flux(orc):
    rng = np.random.default_rng(10)
    dims = (8, 8, 8)
    for _ in range(40):
        d = rng.uniform(0.1, 0.9, 3)
        x0 = np.array([3.0, 4.0, 2.0]) + d
        D = rng.uniform(-1, 1, 3) * np.minimum(d, 1 - d) * 0.99
        assert _check_move(orc, dims, x0, x0 + D, sgn=rng.choice([-1.0, 1.0])) == 1


@pytest.mark.parametrize("ncross", [1, 2, 3])
def test_deposit_cell_crossing_matches_swept_flux(orc, ncross):
    rng = np.random.default_rng(20 + ncross)
    dims = (8, 8, 8)
    done = 0
    while done < 25:
        x0 = np.array([3.0, 4.0, 2.0]) + rng.uniform(0, 1, 3)
        D = rng.uniform(-0.49, 0.49, 3)
        x1 = x0 + D
        nc = int(np.sum(np.floor(x0) != np.floor(x1)))
        if nc != ncross:
            continue
        assert _check_move(orc, dims, x0, x1, sgn=-1.0) == ncross + 1
        done += 1


def test_deposit_continuity_per_node(orc):
    # discrete continuity: div J at each node equals the change of its CIC weight
    rng = np.random.default_rng(30)
    dims = (6, 5, 7)
    n = int(np.prod(dims))
    for _ in range(100):
        x0 = rng.uniform(0, 1, 3) * np.array(dims)
        x1 = x0 + rng.uniform(-0.5, 0.5, 3)
        J, _ = orc.deposit_move(dims, 1.0, x0, x1)
        X = J[:n].reshape(dims[::-1])
        Y = J[n:2 * n].reshape(dims[::-1])
        Z = J[2 * n:].reshape(dims[::-1])
        div = (X - np.roll(X, 1, axis=2)) + (Y - np.roll(Y, 1, axis=1)) + (Z - np.roll(Z, 1, axis=0))
        W = np.zeros(dims[::-1])
        for xx, sgn in ((x1, 1.0), (x0, -1.0)):
            for i in range(int(np.floor(xx[0])) - 1, int(np.floor(xx[0])) + 3):
                for j in range(int(np.floor(xx[1])) - 1, int(np.floor(xx[1])) + 3):
                    for k in range(int(np.floor(xx[2])) - 1, int(np.floor(xx[2])) + 3):
                        w = _ov(xx[0], i) * _ov(xx[1], j) * _ov(xx[2], k)
                        W[k % dims[2], j % dims[1], i % dims[0]] += sgn * w
        assert np.max(np.abs(div - W)) < 1e-14


def test_deposit_exact_plane_endpoints(orc):
    # endpoint exactly on a node plane and a move along a plane: still exact
    dims = (8, 8, 8)
    _check_move(orc, dims, np.array([3.25, 4.5, 2.5]), np.array([4.0, 4.5, 2.5]))
    _check_move(orc, dims, np.array([3.5, 4.0, 2.5]), np.array([3.2, 4.0, 2.9]))
    _check_move(orc, dims, np.array([3.8, 4.8, 2.8]), np.array([4.1, 5.1, 3.1]))  # through an edge
