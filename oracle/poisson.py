"""Exact pseudo-inverse of the pressure Laplacian L = G^T G.

Sec. 4.2 factorises L once with the direct method of Lynch et al.: L is a sum
of Kronecker products of 1-D second-difference matrices, each diagonalised by
its own eigenbasis.  On a uniform grid those eigenbases are known in closed
form: the discrete Fourier basis on a periodic axis and the DCT-II basis on a
Neumann axis (the pressure axis between two walls of either kind).  The 1-D
eigenvalues are (4/h^2) sin^2(pi k / n) and (4/h^2) sin^2(pi k / (2n)).

The zero eigenvalue (constants) is mapped to zero: the result is the
mean-zero solution of L x = b - mean(b).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .mac import PERIODIC, Grid


def eigenvalues_1d(n: int, h: float, bc: int) -> np.ndarray:
    k = np.arange(n)
    if bc == PERIODIC:
        return 4.0 / (h * h) * np.sin(np.pi * k / n) ** 2
    return 4.0 / (h * h) * np.sin(np.pi * k / (2.0 * n)) ** 2


def symbol(g: Grid) -> np.ndarray:
    lam = np.zeros(g.n)
    for a in range(3):
        e = eigenvalues_1d(g.n[a], g.h, g.bc[a])
        shape = [1, 1, 1]
        shape[a] = g.n[a]
        lam = lam + e.reshape(shape)
    return lam


def _forward(g: Grid, x: np.ndarray, workers=None):
    y = x.astype(np.complex128) if any(b == PERIODIC for b in g.bc) else x.copy()
    for a in range(3):
        if g.bc[a] == PERIODIC:
            y = sfft.fft(y, axis=a, workers=workers)
        else:
            if np.iscomplexobj(y):
                y = sfft.dct(y.real, type=2, norm="ortho", axis=a, workers=workers) + \
                    1j * sfft.dct(y.imag, type=2, norm="ortho", axis=a, workers=workers)
            else:
                y = sfft.dct(y, type=2, norm="ortho", axis=a, workers=workers)
    return y


def _inverse(g: Grid, y: np.ndarray, workers=None):
    for a in reversed(range(3)):
        if g.bc[a] == PERIODIC:
            y = sfft.ifft(y, axis=a, workers=workers)
        else:
            if np.iscomplexobj(y):
                y = sfft.idct(y.real, type=2, norm="ortho", axis=a, workers=workers) + \
                    1j * sfft.idct(y.imag, type=2, norm="ortho", axis=a, workers=workers)
            else:
                y = sfft.idct(y, type=2, norm="ortho", axis=a, workers=workers)
    return np.real(y)


def solve_laplacian(g: Grid, b: np.ndarray, workers=None) -> np.ndarray:
    """Mean-zero x with L x = b - mean(b); b has shape g.n."""
    lam = symbol(g)
    y = _forward(g, b, workers)
    lam0 = lam.copy()
    lam0[0, 0, 0] = 1.0
    y = y / lam0
    y[0, 0, 0] = 0.0
    return _inverse(g, y, workers)
