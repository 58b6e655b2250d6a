"""Brute-force evaluation of the same quantities on tiny grids, with no fast transform at all.

TEST INFRASTRUCTURE. Only the tests use it: it pins the transform-based oracle in
``ks_loop.py``.

Fields live as full, centred coefficient arrays c[j + Kx, k + Ks] for |j| <= Kx and
|k| <= Ks, the two-thirds band of Sec. 4.2. Nonlinear terms are formed by the direct
truncated convolution sum (uv)_{j,k} = sum_{j'+j''=j, k'+k''=k} u_{j',k'} v_{j'',k''}.
Space-time integrals are formed by evaluating eq. 2D_Fourier explicitly at the grid points
(x_m, s_n) = (m L / Nx, n / Ns), with exact integer argument reduction
exp(2 pi i ((m j mod Nx) / Nx + (n k mod Ns) / Ns)), and averaging. Pure Python and NumPy
loops only: meant for Nx, Ns <= 16.
"""
from __future__ import annotations

import numpy as np


def limits(Nx, Ns):
    return (Nx - 1) // 3, (Ns - 1) // 3


def from_rfft(uhat: np.ndarray):
    """Full centred band array from the rfft layout; column 0 read through its Hermitian part."""
    Ns, half = uhat.shape
    Nx = 2 * (half - 1)
    Kx, Ks = limits(Nx, Ns)
    c = np.zeros((2 * Kx + 1, 2 * Ks + 1), dtype=np.complex128)
    for j in range(-Kx, Kx + 1):
        for k in range(-Ks, Ks + 1):
            if j > 0:
                v = uhat[k % Ns, j]
            elif j < 0:
                v = np.conj(uhat[(-k) % Ns, -j])
            else:
                v = 0.5 * (uhat[k % Ns, 0] + np.conj(uhat[(-k) % Ns, 0]))
            c[j + Kx, k + Ks] = v
    return c


def to_rfft(c: np.ndarray, Nx: int, Ns: int) -> np.ndarray:
    Kx, Ks = limits(Nx, Ns)
    out = np.zeros((Ns, Nx // 2 + 1), dtype=np.complex128)
    for j in range(0, Kx + 1):
        for k in range(-Ks, Ks + 1):
            out[k % Ns, j] = c[j + Kx, k + Ks]
    return out


def _wn(Kx, Ks, L):
    j = np.arange(-Kx, Kx + 1, dtype=np.float64)
    k = np.arange(-Ks, Ks + 1, dtype=np.float64)
    return (2 * np.pi * j / L)[:, None], (2 * np.pi * k)[None, :]


def conv(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Direct truncated convolution of two centred band arrays."""
    nj, nk = a.shape
    Kx, Ks = (nj - 1) // 2, (nk - 1) // 2
    out = np.zeros_like(a)
    for j in range(-Kx, Kx + 1):
        for k in range(-Ks, Ks + 1):
            acc = 0.0 + 0.0j
            for j1 in range(-Kx, Kx + 1):
                j2 = j - j1
                if abs(j2) > Kx:
                    continue
                for k1 in range(-Ks, Ks + 1):
                    k2 = k - k1
                    if abs(k2) > Ks:
                        continue
                    acc += a[j1 + Kx, k1 + Ks] * b[j2 + Kx, k2 + Ks]
            out[j + Kx, k + Ks] = acc
    return out


def grid_values(c: np.ndarray, Nx: int, Ns: int) -> np.ndarray:
    """Explicit evaluation of eq. 2D_Fourier at every grid point (exact argument reduction)."""
    nj, nk = c.shape
    Kx, Ks = (nj - 1) // 2, (nk - 1) // 2
    out = np.zeros((Ns, Nx), dtype=np.complex128)
    for n in range(Ns):
        for m in range(Nx):
            acc = 0.0 + 0.0j
            for j in range(-Kx, Kx + 1):
                for k in range(-Ks, Ks + 1):
                    phase = ((m * j) % Nx) / Nx + ((n * k) % Ns) / Ns
                    acc += c[j + Kx, k + Ks] * np.exp(2j * np.pi * phase)
            out[n, m] = acc
    return out


def integral(a: np.ndarray, b: np.ndarray, Nx: int, Ns: int, L: float) -> float:
    """int_0^1 int_0^L a b dx ds by the grid average of the explicitly evaluated fields."""
    ga = grid_values(a, Nx, Ns).real
    gb = grid_values(b, Nx, Ns).real
    return float(L * np.mean(ga * gb))


def residual(c, T, L):
    nj, nk = c.shape
    Kx, Ks = (nj - 1) // 2, (nk - 1) // 2
    q, w = _wn(Kx, Ks, L)
    ux = 1j * q * c
    return -(1j * w / T) * c - conv(c, ux) + q ** 2 * c - q ** 4 * c


def grad(c, T, L):
    """G1 = -(1/T) r_s - u r_x + r_xx + r_xxxx in the band."""
    nj, nk = c.shape
    Kx, Ks = (nj - 1) // 2, (nk - 1) // 2
    q, w = _wn(Kx, Ks, L)
    r = residual(c, T, L)
    return -(1j * w / T) * r - conv(c, 1j * q * r) - q ** 2 * r + q ** 4 * r


def all_quantities(uhat, T, L):
    """(r_hat, J, dJ/dT, G1_hat) in rfft layout from the brute-force definitions."""
    Ns, half = uhat.shape
    Nx = 2 * (half - 1)
    Kx, Ks = limits(Nx, Ns)
    c = from_rfft(uhat)
    q, w = _wn(Kx, Ks, L)
    r = residual(c, T, L)
    J = 0.5 * integral(r, r, Nx, Ns, L)
    dT = integral(1j * w * c, r, Nx, Ns, L) / (T * T)
    G = grad(c, T, L)
    return to_rfft(r, Nx, Ns), J, dT, to_rfft(G, Nx, Ns)
