"""Seeded synthetic loop generator shared by the oracle tests, the GPU parity tests and bench.py.

This module holds only random-number draws and array layout. It holds none of the method's
arithmetic: no derivatives, no products, no residual and no transforms.

A loop is l = [u(x, s); T] on x in [0, L), s in [0, 1) (loop space, eq. loop_def, Sec. 2).
Its field is stored as spectral coefficients in the layout of a real two-dimensional
forward-normalised transform of the (Ns, Nx) grid (Sec. 4.2, eq. 2D_Fourier):

    uhat[k mod Ns, j] = u_hat_{j,k},   j = 0 .. Nx/2,   k = -Ns/2 .. Ns/2 - 1,

so row k of the array holds temporal mode k in FFT order and column j holds the non-negative
spatial modes. Negative spatial modes follow from the real-field symmetry
u_hat_{-j,-k} = conj(u_hat_{j,k}).

Spectra follow one recipe throughout:

    u_hat_{j,k} = A * exp(-beta * (|j| + |k|)) * (xi + i*eta) / sqrt(2)

for |j| <= jmax and |k| <= kmax, with xi and eta standard normal. They are drawn from
numpy.random.default_rng(seed) in a fixed order:

1. T0 first.
2. For mixed batches, the shape and L choices.
3. The modes for k = 0 .. kmax, each with j = -jmax .. jmax, on the half plane (k > 0, or
   k = 0 and j > 0).

Each drawn mode is mirrored to its Hermitian partner, and the mean mode is zero.
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence

import numpy as np

__all__ = [
    "LoopSpec",
    "seeded_spectrum",
    "random_loop",
    "config_loops",
    "CONFIGS",
    "random_band_field",
    "random_xi_symmetric_field",
    "from_modes",
    "random_ks_state",
]


@dataclasses.dataclass
class LoopSpec:
    """One synthetic loop: shape, domain length, period and spectrum (rfft layout, complex128)."""

    L: float
    Nx: int
    Ns: int
    T: float
    uhat: np.ndarray  # (Ns, Nx//2+1) complex128
    seed: int

    @property
    def points(self) -> int:
        return self.Nx * self.Ns


def _put(uhat: np.ndarray, j: int, k: int, val: complex) -> None:
    """Store mode (j, k) and its Hermitian partner (-j, -k) into the rfft-layout array."""
    Ns = uhat.shape[0]
    if j > 0:
        uhat[k % Ns, j] = val
    elif j < 0:
        uhat[(-k) % Ns, -j] = np.conj(val)
    else:  # j == 0: both k and -k live in column 0
        uhat[k % Ns, 0] = val
        uhat[(-k) % Ns, 0] = np.conj(val)


def seeded_spectrum(rng: np.random.Generator, Nx: int, Ns: int, jmax: int, kmax: int,
                    amp: float, beta: float) -> np.ndarray:
    """Draw the low-mode spectrum described in the module docstring from ``rng``."""
    if jmax >= Nx // 2 or kmax >= Ns // 2:
        raise ValueError("seeded modes must lie inside the grid")
    uhat = np.zeros((Ns, Nx // 2 + 1), dtype=np.complex128)
    for k in range(0, kmax + 1):
        for j in range(-jmax, jmax + 1):
            if k == 0 and j <= 0:
                continue
            xi, eta = rng.standard_normal(2)
            a = amp * np.exp(-beta * (abs(j) + abs(k)))
            _put(uhat, j, k, a * complex(xi, eta) / np.sqrt(2.0))
    return uhat


def random_loop(seed: int, L: float, Nx: int, Ns: int, jmax: int, kmax: int, amp: float,
                beta: float, T0) -> LoopSpec:
    """T0 is a number or a (lo, hi) pair for a uniform draw (drawn first)."""
    rng = np.random.default_rng(seed)
    if isinstance(T0, tuple):
        T = float(rng.uniform(T0[0], T0[1]))
    else:
        T = float(T0)
    uhat = seeded_spectrum(rng, Nx, Ns, jmax, kmax, amp, beta)
    return LoopSpec(L=float(L), Nx=Nx, Ns=Ns, T=T, uhat=uhat, seed=seed)


# The five benchmark workloads. Seeds: workload c, loop i -> 1000*c + i.
CONFIGS = {
    1: dict(name="plain-32x32", L=22.0, Nx=32, Ns=32, jmax=4, kmax=3, amp=0.5, beta=0.3,
            T0=20.0, loops=1, scheme="explicit", dtau=1e-4, steps=2000),
    2: dict(name="plain-64x128", L=22.0, Nx=64, Ns=128, jmax=8, kmax=8, amp=0.5, beta=0.2,
            T0=(30.0, 60.0), loops=1, scheme="imex", dtau=5e-5, steps=20000),
    3: dict(name="autograd-64x256", L=39.0, Nx=64, Ns=256, jmax=8, kmax=8, amp=0.5, beta=0.2,
            T0=(30.0, 60.0), loops=1, scheme="imex", dtau=5e-5, steps=0),
    4: dict(name="batched-ragged-256", L=(22.0, 39.0), Nx=(32, 64), Ns=(64, 128, 256, 512),
            jmax=4, kmax=3, amp=0.5, beta=0.3, T0=(20.0, 80.0), loops=256, scheme="imex",
            dtau=5e-5, steps=5000),
    5: dict(name="batched-256x1024", L=100.0, Nx=256, Ns=1024, jmax=24, kmax=32, amp=0.5,
            beta=0.15, T0=(50.0, 150.0), loops=64, scheme="imex", dtau=5e-5, steps=2000),
}


def config_loops(c: int, nloops: int | None = None) -> List[LoopSpec]:
    """The seeded loops of workload ``c`` (optionally only the first ``nloops``)."""
    cfg = CONFIGS[c]
    n = cfg["loops"] if nloops is None else nloops
    out = []
    for i in range(n):
        seed = 1000 * c + i
        if c == 4:
            rng = np.random.default_rng(seed)
            T = float(rng.uniform(*cfg["T0"]))
            Nx = int(rng.choice(cfg["Nx"]))
            Ns = int(rng.choice(cfg["Ns"]))
            L = float(rng.choice(cfg["L"]))
            uhat = seeded_spectrum(rng, Nx, Ns, cfg["jmax"], cfg["kmax"], cfg["amp"], cfg["beta"])
            out.append(LoopSpec(L=L, Nx=Nx, Ns=Ns, T=T, uhat=uhat, seed=seed))
        else:
            out.append(random_loop(seed, cfg["L"], cfg["Nx"], cfg["Ns"], cfg["jmax"], cfg["kmax"],
                                   cfg["amp"], cfg["beta"], cfg["T0"]))
    return out


def random_band_field(rng: np.random.Generator, Nx: int, Ns: int, jmax: int | None = None,
                      kmax: int | None = None, scale: float = 1.0, zero_mean: bool = False
                      ) -> np.ndarray:
    """Random real field with all modes |j| <= jmax, |k| <= kmax filled with O(scale) values.

    Defaults fill the whole two-thirds band (|j| <= (Nx-1)//3, |k| <= (Ns-1)//3).
    """
    jmax = (Nx - 1) // 3 if jmax is None else jmax
    kmax = (Ns - 1) // 3 if kmax is None else kmax
    uhat = np.zeros((Ns, Nx // 2 + 1), dtype=np.complex128)
    for k in range(0, kmax + 1):
        for j in range(-jmax, jmax + 1):
            if k == 0 and j < 0:
                continue
            xi, eta = rng.standard_normal(2)
            if k == 0 and j == 0:
                if not zero_mean:
                    uhat[0, 0] = scale * xi
                continue
            _put(uhat, j, k, scale * complex(xi, eta) / np.sqrt(2.0))
    return uhat


def random_xi_symmetric_field(rng: np.random.Generator, Nx: int, Ns: int,
                              jmax: int | None = None, kmax: int | None = None,
                              scale: float = 1.0) -> np.ndarray:
    """Random field invariant under (x, s) -> (-x, s), u -> -u (loop symmetry Xi, Sec. 4.1).

    u odd in x means u_hat_{-j,k} = -u_hat_{j,k}; together with reality this gives
    u_hat_{j,k} = -conj(u_hat_{j,-k}), so each mode is drawn for k >= 0 and j > 0 and
    mirrored, and column j = 0 is zero.
    """
    jmax = (Nx - 1) // 3 if jmax is None else jmax
    kmax = (Ns - 1) // 3 if kmax is None else kmax
    uhat = np.zeros((Ns, Nx // 2 + 1), dtype=np.complex128)
    for j in range(1, jmax + 1):
        for k in range(0, kmax + 1):
            xi, eta = rng.standard_normal(2)
            v = scale * complex(xi, eta) / np.sqrt(2.0)
            if k == 0:
                v = complex(0.0, v.imag)  # u_hat_{j,0} = -conj(u_hat_{j,0}) => purely imaginary
                uhat[0, j] = v
            else:
                uhat[k % Ns, j] = v
                uhat[(-k) % Ns, j] = -np.conj(v)
    return uhat


def random_ks_state(rng: np.random.Generator, Nx: int, jmax: int | None = None, scale: float = 1.0,
                    odd: bool = False) -> np.ndarray:
    """Random instantaneous KS field (one time) in the rfft layout (Nx//2 + 1,), zero mean, modes
    1 <= j <= jmax (default the two-thirds band) drawn as scale (xi + i eta) / sqrt(2) in order
    of j. With odd=True the field is odd in x (centre-symmetric, eq. KS_sym): each mode is
    i * scale * xi, purely imaginary."""
    jmax = (Nx - 1) // 3 if jmax is None else jmax
    u = np.zeros(Nx // 2 + 1, dtype=np.complex128)
    for j in range(1, jmax + 1):
        if odd:
            u[j] = 1j * scale * rng.standard_normal()
        else:
            xi, eta = rng.standard_normal(2)
            u[j] = scale * complex(xi, eta) / np.sqrt(2.0)
    return u


def from_modes(Nx: int, Ns: int, modes: Sequence[tuple]) -> np.ndarray:
    """Build an rfft-layout spectrum from explicit (j, k, value) triples plus Hermitian partners."""
    uhat = np.zeros((Ns, Nx // 2 + 1), dtype=np.complex128)
    for j, k, v in modes:
        _put(uhat, j, k, complex(v))
    return uhat
