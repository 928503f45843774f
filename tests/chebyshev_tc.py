"""Brute-force linear stability of circular Couette flow to axisymmetric
disturbances, independent of the oracle (different variables, different
discretisation): Chebyshev collocation of the classical two-field form

    lam (D D_* - alpha^2) u_r = nu (D D_* - alpha^2)^2 u_r - 2 alpha^2 (V / r) u_t
    lam u_t                   = nu (D D_* - alpha^2) u_t - (V' + V / r) u_r

obtained from the linearised primitive equations by eliminating the pressure
and the axial velocity (continuity), with u_r = D u_r = u_t = 0 at both walls,
about the base flow V(r) = A r + B / r.  Lengths in units of the gap, inner
wall speed 1, nu = 1 / Re.
"""

import numpy as np
from scipy.linalg import eig


def cheb(n):
    """Chebyshev differentiation matrix and Gauss--Lobatto points on [-1, 1]."""
    x = np.cos(np.pi * np.arange(n + 1) / n)
    c = np.ones(n + 1)
    c[0] = c[-1] = 2.0
    c *= (-1.0) ** np.arange(n + 1)
    X = np.tile(x, (n + 1, 1)).T
    dX = X - X.T
    D = np.outer(c, 1.0 / c) / (dX + np.eye(n + 1))
    D -= np.diag(D.sum(axis=1))
    return D, x


def growth_rate(zeta, re, alpha, n=40, w_outer=0.0):
    """Largest real part of the eigenvalues."""
    ri = zeta / (1 - zeta)
    ro = 1.0 / (1 - zeta)
    D, x = cheb(n)
    r = ri + (x + 1) * (ro - ri) / 2
    D = D * 2 / (ro - ri)
    I = np.eye(n + 1)
    R = np.diag(r)
    Rinv = np.diag(1 / r)
    a = (w_outer * ro - ri) / (ro**2 - ri**2)
    b = ri - a * ri**2
    V = a * r + b / r
    dV = a - b / r**2
    nu = 1.0 / re
    Ds = D + Rinv                     # D_*
    L = D @ Ds - alpha**2 * I         # D D_* - alpha^2
    N = n + 1
    A = np.zeros((2 * N, 2 * N), dtype=complex)
    B = np.zeros((2 * N, 2 * N), dtype=complex)
    A[:N, :N] = nu * L @ L
    A[:N, N:] = -2 * alpha**2 * np.diag(V / r)
    B[:N, :N] = L
    A[N:, :N] = -np.diag(dV + V / r)
    A[N:, N:] = nu * L
    B[N:, N:] = I
    # boundary rows: u_r = 0 and D u_r = 0 at both walls, u_t = 0 at both walls
    for row, vec in ((0, I[0]), (N - 1, I[N - 1]), (1, D[0]), (N - 2, D[N - 1])):
        A[row] = 0
        B[row] = 0
        A[row, :N] = vec
    for row in (N, 2 * N - 1):
        A[row] = 0
        B[row] = 0
        A[row, row] = 1
    lam = eig(A, B, right=False)
    lam = lam[np.isfinite(lam) & (np.abs(lam) < 1e6)]
    return np.max(lam.real)
