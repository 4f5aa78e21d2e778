"""Shared helpers for the oracle pins: golden-file readers and independent
constructions (exact rationals, Kronecker-sum matrices).  Nothing here
imports the oracle or the HIP library."""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def golden_coefficients():
    """c_0..c_4 as Fractions from the published table."""
    c = [None] * 5
    for m, num, den in read_table("coefficients_8th_order.txt"):
        c[int(m)] = Fraction(int(num), int(den))
    return c


def second_derivative_matrix(n: int, h: float, c) -> np.ndarray:
    """Dense n x n matrix of the 1-D 8th-order second derivative with a zero
    ghost layer (rows simply lose the taps that fall outside)."""
    D = np.zeros((n, n))
    cf = [float(x) for x in c]
    for i in range(n):
        D[i, i] = cf[0]
        for m in range(1, 5):
            if i + m < n:
                D[i, i + m] = cf[m]
            if i - m >= 0:
                D[i, i - m] = cf[m]
    return D / (h * h)


def kron_laplacian(nz: int, ny: int, nx: int, h, c):
    """3-D Laplacian on the flattened [z][y][x] interior as a Kronecker sum
    of 1-D operators (scipy sparse)."""
    import scipy.sparse as sp

    dx, dy, dz = h
    Dx = sp.csr_matrix(second_derivative_matrix(nx, dx, c))
    Dy = sp.csr_matrix(second_derivative_matrix(ny, dy, c))
    Dz = sp.csr_matrix(second_derivative_matrix(nz, dz, c))
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    return (sp.kron(Dz, sp.kron(Iy, Ix)) + sp.kron(Iz, sp.kron(Dy, Ix))
            + sp.kron(Iz, sp.kron(Iy, Dx))).tocsr()


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))
