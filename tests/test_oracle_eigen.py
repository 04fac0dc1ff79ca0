"""Pins of the oracle's MHD flux and characteristic system (arXiv:1808.10633
Sec. 2.1: Roe-type decoupling of the 8 PDEs; eigenvectors deferred by the
paper).  Checked against invariants: L R = I, A R = R Lambda with A the
finite-difference Jacobian of the oracle's own flux, eigenvalues of A from
numpy, the Euler limit, and rotational consistency of the flux."""
import math

import numpy as np
import pytest

G = 5.0 / 3.0


def fd_jacobian(orc, U, gamma=G, direction=0):
    """Central-difference Jacobian dF/dU along axis 0 (Bn column left zero)."""
    A = np.zeros((8, 8))
    for c in range(8):
        if c == 4 + direction:
            continue
        h = 1e-6 * max(1.0, abs(U[c]))
        up = U.copy(); up[c] += h
        um = U.copy(); um[c] -= h
        A[:, c] = (orc.flux(up, direction, gamma) - orc.flux(um, direction, gamma)) / (2 * h)
    return A


def states():
    rng = np.random.default_rng(11)
    out = []
    for _ in range(30):
        out.append(np.array([rng.uniform(0.3, 3), *rng.normal(size=3),
                             *rng.normal(size=3), rng.uniform(0.2, 3)]))
    s2 = math.sqrt(0.6)
    out += [
        np.array([1.0, 0.3, 0.1, -0.2, 0.8, 0.0, 0.0, 0.7]),        # B_t = 0
        np.array([1.0, 0.3, 0.1, -0.2, 0.0, 0.6, -0.4, 0.7]),       # B_n = 0
        np.array([1.0, 0.3, 0.1, -0.2, 0.0, 0.0, 0.0, 0.7]),        # B = 0 (Euler)
        np.array([1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.6]),         # triple point a = c_A
        np.array([1.0, 0.0, 0.0, 0.0, 1.0, 1e-9, 0.0, 0.6]),        # near triple point
        np.array([1.0, 0.0, 0.0, 0.0, 1.0, 1e-7, 2e-7, 0.6 + 1e-8]),
        np.array([2.0, 0.1, 0.0, 0.0, 2.0, 1e-13, -1e-13, 0.3]),     # tiny B_t, a < c_A
        np.array([1.0, 0.0, 0.0, 0.0, s2, 0.0, 0.0, 0.6]),          # a > c_A, B_t = 0
        np.array([1.0, -2.0, 1.0, 0.5, -0.9, 0.3, 0.2, 1e-3]),      # cold, B_n < 0
        np.array([1e-3, 0.0, 0.0, 0.0, 0.1, 0.1, 0.0, 10.0]),       # hot, light
    ]
    return out


@pytest.mark.parametrize("k", range(40))
def test_left_right_inverse(orc, k):
    W = states()[k]
    lam, L, R = orc.eigensystem(W, G)
    assert np.abs(L @ R - np.eye(8)).max() < 1e-12
    # and the vectors stay well conditioned near degeneracies
    assert np.linalg.cond(R) < 1e8


@pytest.mark.parametrize("k", range(40))
def test_right_eigenvectors_of_fd_jacobian(orc, k):
    W = states()[k]
    U = orc.prim_to_cons(W, G)
    lam, L, R = orc.eigensystem(W, G)
    A = fd_jacobian(orc, U)
    scale = np.abs(A).max() * np.abs(R).max() + 1.0
    res = np.abs(A @ R[:, :7] - R[:, :7] * lam[:7]).max() / scale
    assert res < 2e-7, res
    # left eigenvectors: L A = Lambda L
    resl = np.abs(L[:7] @ A - lam[:7, None] * L[:7]).max() / (np.abs(A).max() * np.abs(L).max() + 1.0)
    assert resl < 2e-7, resl


@pytest.mark.parametrize("k", range(40))
def test_eigenvalues_match_numpy(orc, k):
    W = states()[k]
    U = orc.prim_to_cons(W, G)
    lam, L, R = orc.eigensystem(W, G)
    A = fd_jacobian(orc, U)
    sub = [0, 1, 2, 3, 5, 6, 7]
    ev = np.sort(np.linalg.eigvals(A[np.ix_(sub, sub)]).real)
    assert np.allclose(ev, np.sort(lam[:7]), atol=1e-5 * (1 + np.abs(lam).max()))


def test_euler_limit(orc):
    # B = 0: the fast pair must be the Euler acoustic waves v -+ a and the
    # fast right eigenvectors the acoustic ones (1, v-+a, vt, H-+v a).
    g = 1.4
    W = np.array([1.3, 0.4, -0.2, 0.1, 0, 0, 0, 0.9])
    lam, L, R = orc.eigensystem(W, g)
    a = math.sqrt(g * W[7] / W[0])
    assert abs(lam[0] - (W[1] - a)) < 1e-14 and abs(lam[6] - (W[1] + a)) < 1e-14
    U = orc.prim_to_cons(W, g)
    H = (U[7] + W[7]) / W[0]
    for col, sg in ((0, -1), (6, 1)):
        r = R[:, col] / R[0, col]
        want = np.array([1, W[1] + sg * a, W[2], W[3], 0, 0, 0, H + sg * W[1] * a])
        assert np.abs(r - want).max() < 1e-13


def test_flux_rotational_consistency(orc):
    # F_y(U) equals F_x of the cyclically relabelled state, relabelled back.
    rng = np.random.default_rng(3)
    for _ in range(20):
        U = orc.prim_to_cons(np.array([rng.uniform(0.5, 2), *rng.normal(size=6), rng.uniform(0.5, 2)]))
        for d in (1, 2):
            t1, t2 = (d + 1) % 3, (d + 2) % 3
            perm = [0, 1 + d, 1 + t1, 1 + t2, 4 + d, 4 + t1, 4 + t2, 7]
            Fd = orc.flux(U, d)
            Fx = orc.flux(U[perm], 0)
            back = np.zeros(8)
            back[perm] = Fx
            assert np.abs(Fd - back).max() < 1e-14 * (1 + np.abs(Fd).max())


def test_wave_speeds_closed_forms(orc):
    # Parallel and perpendicular propagation have textbook speeds:
    # along B: c_f = max(a, c_A), c_s = min(a, c_A); across B: c_f = sqrt(a^2+b^2).
    g = G
    rho, p, Bx = 1.7, 0.8, 1.3
    a = math.sqrt(g * p / rho)
    cA = Bx / math.sqrt(rho)
    U = orc.prim_to_cons(np.array([rho, 0, 0, 0, Bx, 0, 0, p]), g)
    cf, ca, cs = orc.wave_speeds(U, 0, g)
    assert abs(cf - max(a, cA)) < 1e-14 and abs(cs - min(a, cA)) < 1e-14 and abs(ca - cA) < 1e-14
    cf, ca, cs = orc.wave_speeds(U, 1, g)
    assert abs(cf - math.sqrt(a * a + cA * cA)) < 1e-14 and cs == 0.0 and ca == 0.0


def test_interface_flux_consistency(orc):
    # A uniform stencil has no differences, so eq. (1) returns the central
    # term, and the back-projection (R L = I) returns the physical flux.
    rng = np.random.default_rng(8)
    for _ in range(10):
        U = orc.prim_to_cons(np.array([rng.uniform(0.5, 2), *rng.normal(size=6), rng.uniform(0.5, 2)]))
        Fh = orc.interface_flux(np.tile(U, (6, 1)))
        F = orc.flux(U, 0)
        assert np.abs(Fh - F).max() < 1e-13 * (1 + np.abs(F).max())
        assert Fh[4] == 0.0 or abs(Fh[4]) < 1e-15
