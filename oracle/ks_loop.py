"""FP64 CPU oracle for one fictitious-time step of the Kuramoto-Sivashinsky loop dynamics.

TEST INFRASTRUCTURE. This module is the parity reference for the HIP path. Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it. The product
path never calls it, and it shares no code with the HIP kernels or their host library.

What is computed, following Azimi, Ashtari & Schneider, "Adjoint-based variational method
for constructing periodic orbits of high-dimensional chaotic systems" (arXiv:2007.06427):

* loop l = [u(x, s); T] on x in [0, L), s in [0, 1), both periodic   (Sec. 2, eq. loop_def)
* residual  r = -(1/T) u_s - u u_x - u_xx - u_xxxx                    (Sec. 4.1, eq. KS_R)
* cost      J = 1/2 * int_0^1 int_0^L r^2 dx ds   (half the paper's eq. cost_function, so that
            the flow of eq. KS_G is exactly the negative gradient of J)
* dJ/dT   = int int (1/T^2) u_s r dx ds          (second row of eq. KS_L_dagger, App. B)
* G_1     = -(1/T) r_s - u r_x + r_xx + r_xxxx    (first row of eq. KS_G)
* G_2     = -dJ/dT                                (second row of eq. KS_G)
* step      semi-implicit Euler for u (linear terms implicit, the rest explicit) or explicit
            Euler, explicit Euler for T                                (Sec. 4.2)

Discretisation (Sec. 4.2, eq. 2D_Fourier): Fourier in x and s, forward-normalised,
u(x_m, s_n) = sum_{j,k} u_hat_{j,k} exp(2 pi i (m j / Nx + n k / Ns)). Derivatives act in
spectral space (d/dx -> i q_j, q_j = 2 pi j / L; d/ds -> i omega_k, omega_k = 2 pi k).
Products are pointwise on the (Ns, Nx) grid. Every result is truncated to the two-thirds band
|j| <= (Nx-1)//3, |k| <= (Ns-1)//3, in both directions. Space-time integrals are taken the
way the paper takes them: form the integrand on the grid, transform, and multiply the (0, 0)
mode by L (Sec. 4.2).

Because every product here is of two band-limited fields, the grid products are free of
aliasing inside the band. The results are therefore the exact Galerkin-truncated values.

Arrays use the layout of ``numpy.fft.rfft2(u, norm="forward")`` for a real (Ns, Nx) grid:
shape (Ns, Nx//2 + 1), row k in FFT order, column j = 0 .. Nx/2. Column 0 of an input is read
through its Hermitian part: this is the field that the real-valued inverse transform
produces.

numpy.fft (pocketfft, double precision) is used as a library primitive for the transforms.
The brute-force module in this package pins it with explicit DFT sums and direct
convolutions.
"""
from __future__ import annotations

import numpy as np

EXPLICIT = 0
IMEX = 1


# --------------------------------------------------------------------------------------------
# grid, band and spectral operators (Sec. 4.2)
# --------------------------------------------------------------------------------------------
def band_limits(Nx: int, Ns: int):
    """Largest retained |j| and |k| under the two-thirds rule (Sec. 4.2)."""
    return (Nx - 1) // 3, (Ns - 1) // 3


def _shape(a: np.ndarray):
    Ns, half = a.shape
    return 2 * (half - 1), Ns


def wavenumbers(L: float, Nx: int, Ns: int):
    """q_j = 2 pi j / L for the rfft columns and omega_k = 2 pi k for the FFT-ordered rows."""
    j = np.arange(Nx // 2 + 1, dtype=np.float64)
    k = np.fft.fftfreq(Ns, d=1.0 / Ns)  # exact integers 0..Ns/2-1, -Ns/2..-1
    q = 2.0 * np.pi * j / L
    omega = 2.0 * np.pi * k
    return q[None, :], omega[:, None]


def band_mask(Nx: int, Ns: int) -> np.ndarray:
    Kx, Ks = band_limits(Nx, Ns)
    j = np.arange(Nx // 2 + 1)
    k = np.fft.fftfreq(Ns, d=1.0 / Ns)
    return (np.abs(k)[:, None] <= Ks) & (j[None, :] <= Kx)


def project(vhat: np.ndarray) -> np.ndarray:
    """Two-thirds-rule truncation in x and s (Sec. 4.2)."""
    Nx, Ns = _shape(vhat)
    return np.where(band_mask(Nx, Ns), vhat, 0.0 + 0.0j)


def hermitian_column0(vhat: np.ndarray) -> np.ndarray:
    """Replace column j = 0 by its Hermitian part, (v_k + conj(v_{-k})) / 2.

    A real field has u_hat_{0,-k} = conj(u_hat_{0,k}). The Hermitian part is the spectrum of
    the real field that the inverse real transform produces from column 0.
    """
    out = np.array(vhat, dtype=np.complex128, copy=True)
    c = out[:, 0]
    cm = np.conj(np.roll(c[::-1], 1))  # conj(c[-k mod Ns])
    out[:, 0] = 0.5 * (c + cm)
    return out


def canonical(uhat: np.ndarray) -> np.ndarray:
    """The loop's field as a band-limited real spectrum: project and enforce reality."""
    return hermitian_column0(project(uhat))


def to_grid(vhat: np.ndarray) -> np.ndarray:
    """u(x_m, s_n) on the (Ns, Nx) grid, eq. 2D_Fourier (forward-normalised inverse)."""
    Nx, Ns = _shape(vhat)
    return np.fft.irfft2(vhat, s=(Ns, Nx), norm="forward")


def from_grid(v: np.ndarray) -> np.ndarray:
    """Spectral coefficients of a real grid field (inverse of ``to_grid``)."""
    return np.fft.rfft2(v, norm="forward")


def d_x(vhat, L):
    Nx, Ns = _shape(vhat)
    q, _ = wavenumbers(L, Nx, Ns)
    return 1j * q * vhat


def d_s(vhat, L):
    Nx, Ns = _shape(vhat)
    _, omega = wavenumbers(L, Nx, Ns)
    return 1j * omega * vhat


def d_xx(vhat, L):
    return d_x(d_x(vhat, L), L)


def d_xxxx(vhat, L):
    return d_xx(d_xx(vhat, L), L)


def product(ahat: np.ndarray, bhat: np.ndarray) -> np.ndarray:
    """Pseudo-spectral product: pointwise on the grid, back to spectral space, truncated."""
    return project(from_grid(to_grid(ahat) * to_grid(bhat)))


def space_time_integral(v: np.ndarray, L: float) -> float:
    """int_0^1 int_0^L v dx ds of a grid field: the (0, 0) Fourier mode times L (Sec. 4.2)."""
    return float(np.real(from_grid(v)[0, 0]) * L)


def inner(ahat, bhat, L, a2: float = 0.0, b2: float = 0.0) -> float:
    """<q, q'> = int int q1 q1' dx ds + q2 q2' (eq. inner_product_definition), on the grid."""
    return space_time_integral(to_grid(ahat) * to_grid(bhat), L) + a2 * b2


def lam(T: float, L: float, Nx: int, Ns: int) -> np.ndarray:
    """lambda_{j,k} = -(2 pi k / T)^2 - q^8 + 2 q^6 - q^4: the linear part of the flow (Sec. 4.2)."""
    q, omega = wavenumbers(L, Nx, Ns)
    return -(omega / T) ** 2 - q ** 8 + 2.0 * q ** 6 - q ** 4


# --------------------------------------------------------------------------------------------
# O1 residual, O2 cost, O3 dJ/dT, O4 adjoint gradient (Sec. 4.1, App. B)
# --------------------------------------------------------------------------------------------
def residual(uhat: np.ndarray, T: float, L: float) -> np.ndarray:
    """r = -(1/T) u_s - u u_x - u_xx - u_xxxx (eq. KS_R), truncated to the band."""
    u = canonical(uhat)
    r = -(1.0 / T) * d_s(u, L) - product(u, d_x(u, L)) - d_xx(u, L) - d_xxxx(u, L)
    return project(r)


def cost(uhat: np.ndarray, T: float, L: float) -> float:
    """J = 1/2 int int r^2 dx ds (half of eq. cost_function)."""
    r = to_grid(residual(uhat, T, L))
    return 0.5 * space_time_integral(r * r, L)


def dJdT(uhat: np.ndarray, T: float, L: float) -> float:
    """dJ/dT = int int (1/T^2) u_s r dx ds (eq. KS_L_dagger, second row; App. B)."""
    u = canonical(uhat)
    r = to_grid(residual(u, T, L))
    u_s = to_grid(d_s(u, L))
    return space_time_integral(u_s * r / (T * T), L)


def adjoint_grad(uhat: np.ndarray, T: float, L: float):
    """Return (G1_hat, dJ/dT, J) with G1 = -(1/T) r_s - u r_x + r_xx + r_xxxx (eq. KS_G).

    The period's flow component is G_2 = -dJ/dT.
    """
    u = canonical(uhat)
    r = residual(u, T, L)
    G = -(1.0 / T) * d_s(r, L) - product(u, d_x(r, L)) + d_xx(r, L) + d_xxxx(r, L)
    rg = to_grid(r)
    J = 0.5 * space_time_integral(rg * rg, L)
    dT = space_time_integral(to_grid(d_s(u, L)) * rg / (T * T), L)
    return project(G), dT, J


def expanded_grad(uhat: np.ndarray, T: float, L: float):
    """The paper's own evaluation of the flow (Sec. 4.2, eq. KS_G_1): G_1 = G_1L + G_1NL with
        G_1L  = (1/T^2) u_ss - u_xxxxxxxx - 2 u_xxxxxx - u_xxxx = lambda u_hat,
        G_1NL = -5 u_xxxx u_x - 10 u_xxx u_xx - 3 u_xx u_x + u^2 u_xx + u u_x^2
                + (2u/T) u_xs + (1/T) u_x u_s,
    the derivatives formed in spectral space, the fields on the grid, the products pointwise
    there, and the sum transformed back and truncated to the band. dJ/dT = int int (1/T^2) u_s r
    and J = 1/2 int int r^2 take their integrands on the grid, with r = -(1/T) u_s - u u_x - u_xx
    - u_xxxx formed pointwise there (Sec. 4.2). Returns (G1_hat, dJ/dT, J).

    The cubic products are not free of aliasing under the two-thirds rule, and no intermediate
    is truncated, so this G differs from adjoint_grad's by truncation and aliasing errors; for
    fields of modes |j| <= Kx/3, |k| <= Ks/3 every product stays in the band and the two agree."""
    u = canonical(uhat)
    Nx, Ns = _shape(u)
    g = to_grid
    U, Ux, Uxx = g(u), g(d_x(u, L)), g(d_xx(u, L))
    Uxxx, Uxxxx = g(d_x(d_xx(u, L), L)), g(d_xxxx(u, L))
    Us, Uxs = g(d_s(u, L)), g(d_x(d_s(u, L), L))
    nl = (-5.0 * Uxxxx * Ux - 10.0 * Uxxx * Uxx - 3.0 * Uxx * Ux + U * U * Uxx + U * Ux * Ux
          + (2.0 / T) * U * Uxs + (1.0 / T) * Ux * Us)
    G = lam(T, L, Nx, Ns) * u + project(from_grid(nl))
    r = -(1.0 / T) * Us - U * Ux - Uxx - Uxxxx
    return project(G), space_time_integral(Us * r / (T * T), L), 0.5 * space_time_integral(r * r, L)


def step_expanded(uhat: np.ndarray, T: float, L: float, dtau: float, scheme: int = EXPLICIT, nsteps: int = 1):
    """The paper's step on eq. KS_G_1 (Sec. 4.2): u_hat' = (u_hat + dtau G_1NL) / (1 - dtau lambda)
    (IMEX) or u_hat + dtau G_1 (explicit), T' = T - dtau dJ/dT, from expanded_grad."""
    u = canonical(uhat)
    Nx, Ns = _shape(u)
    J_hist = np.zeros(nsteps)
    for i in range(nsteps):
        G, dT, J = expanded_grad(u, T, L)
        J_hist[i] = J
        lm = lam(T, L, Nx, Ns)
        if scheme == EXPLICIT:
            u_new = u + dtau * G
        elif scheme == IMEX:
            u_new = (u + dtau * (G - lm * u)) / (1.0 - dtau * lm)
        else:
            raise ValueError("scheme must be EXPLICIT (0) or IMEX (1)")
        T = T - dtau * dT
        u = project(u_new)
    return u, T, J_hist


def xi_project(uhat: np.ndarray) -> np.ndarray:
    """Orthogonal projection onto centre-symmetric loops (Sec. 3, eq. KS_loop_sym): the part of
    u invariant under Xi: u(x, s) -> -u(-x, s), i.e. (u + Xi u) / 2, which in Fourier space is
    u_hat_{j,k} -> (u_hat_{j,k} - conj u_hat_{j,-k}) / 2 (column 0 and the Nyquist column, for
    which u_hat_{-j} is the column itself, become 0)."""
    u = canonical(uhat)
    Nx, Ns = _shape(u)
    k_neg = (-np.arange(Ns)) % Ns
    p = 0.5 * (u - np.conj(u[k_neg, :]))
    p[:, 0] = 0.0
    return project(p)


def step(uhat: np.ndarray, T: float, L: float, dtau: float, scheme: int = EXPLICIT,
         nsteps: int = 1):
    """Advance the loop by ``nsteps`` fictitious-time steps (Sec. 4.2).

    Explicit:  u <- u + dtau * G_1.
    IMEX:      the linear terms lambda u_hat are implicit and the rest N = G_1 - lambda u_hat
               is explicit, so (u' - u) / dtau = lambda u' + N(u).
    Period:    T <- T + dtau * G_2 = T - dtau * dJ/dT (explicit Euler).

    Both updates use the state at the start of the step. Returns (uhat, T, J_hist), where
    J_hist[i] is the cost at the start of step i.
    """
    u = canonical(uhat)
    Nx, Ns = _shape(u)
    J_hist = np.zeros(nsteps)
    for i in range(nsteps):
        G, dT, J = adjoint_grad(u, T, L)
        J_hist[i] = J
        if scheme == EXPLICIT:
            u_new = u + dtau * G
        elif scheme == IMEX:
            lm = lam(T, L, Nx, Ns)
            nonlin = G - lm * u
            u_new = (u + dtau * nonlin) / (1.0 - dtau * lm)
        else:
            raise ValueError("scheme must be EXPLICIT (0) or IMEX (1)")
        T = T - dtau * dT
        u = project(u_new)
    return u, T, J_hist


# --------------------------------------------------------------------------------------------
# test-only operators: directional derivative and its adjoint (Sec. 3, App. B)
# --------------------------------------------------------------------------------------------
def directional_derivative(uhat, T, L, v1hat, v2: float) -> np.ndarray:
    """First component of L(l; v): (v2/T^2) u_s - (1/T) v1_s - (u v1)_x - v1_xx - v1_xxxx (App. B)."""
    u = canonical(uhat)
    v1 = canonical(v1hat)
    out = (v2 / (T * T)) * d_s(u, L) - (1.0 / T) * d_s(v1, L) - d_x(product(u, v1), L) \
        - d_xx(v1, L) - d_xxxx(v1, L)
    return project(out)


def adjoint_operator(uhat, T, L, what: np.ndarray):
    """L^dagger(l; [w; 0]) = [(1/T) w_s + u w_x - w_xx - w_xxxx ; int int (1/T^2) u_s w] (eq. KS_L_dagger)."""
    u = canonical(uhat)
    w = canonical(what)
    a1 = (1.0 / T) * d_s(w, L) + product(u, d_x(w, L)) - d_xx(w, L) - d_xxxx(w, L)
    a2 = space_time_integral(to_grid(d_s(u, L)) * to_grid(w) / (T * T), L)
    return project(a1), a2


def autograd_grad(uhat, T, L):
    """Gradient of J with respect to the rfft-layout coefficients in the complex convention
    grad = dJ/dRe + i dJ/dIm, under the reading that column 0 enters through its Hermitian
    part and out-of-band inputs are ignored.

    Derived from J's definition: J depends on u_hat_{j,k} with j >= 1 through both (j,k) and
    its partner (-j,-k), which gives weight 2 L. In column 0 a coefficient and its partner
    share the one array column, which gives weight L. Since G_1 = -grad_L2 J, the result is
    -w_j L G1_hat in the band and 0 elsewhere. Returns (grad_uhat, dJ/dT).
    """
    G, dT, _ = adjoint_grad(uhat, T, L)
    Nx, Ns = _shape(G)
    w = np.full(Nx // 2 + 1, 2.0)
    w[0] = 1.0
    return -w[None, :] * L * G, dT
