"""Brute-force evaluation of Cartesian Gaussian ERIs, independent of any
recurrence: the Coulomb kernel is written as a Gaussian transform,

    1/r = (2/sqrt(pi)) * int_0^inf exp(-t^2 r^2) dt,

so an ERI of monomial Gaussians factorises, for each t, into three 2D Gaussian
integrals of polynomials (one per Cartesian axis).  Each 2D integral is done
exactly by tensor Gauss-Hermite quadrature after completing the square; the
remaining 1D integral over t is mapped to u in [0,1) by t = sqrt(rho) u/sqrt(1-u^2)
(rho = pq/(p+q)), where the integrand is smooth, and done by Gauss-Legendre.
The long-range operator erf(omega r)/r is the same transform cut at t = omega.

Used only by the oracle pins.
"""
from __future__ import annotations

import numpy as np

_GH_X, _GH_W = np.polynomial.hermite.hermgauss(12)
_GL_X, _GL_W = np.polynomial.legendre.leggauss(80)
_GL_U = 0.5 * (_GL_X + 1.0)
_GL_WU = 0.5 * _GL_W


def _axis_integral(i, j, k, l, a, b, c, d, A, B, C, D, t):
    """int int (x1-A)^i (x1-B)^j e^{-a(x1-A)^2 - b(x1-B)^2}
               (x2-C)^k (x2-D)^l e^{-c(x2-C)^2 - d(x2-D)^2} e^{-t^2 (x1-x2)^2} dx1 dx2"""
    # exponent = -[x1 x2] M [x1 x2]^T + 2 h.[x1 x2] - const
    M = np.array([[a + b + t * t, -t * t], [-t * t, c + d + t * t]])
    h = np.array([a * A + b * B, c * C + d * D])
    const = a * A * A + b * B * B + c * C * C + d * D * D
    mu = np.linalg.solve(M, h)
    c0 = -const + h @ mu
    R = np.linalg.cholesky(M)            # M = R R^T
    Rinv_T = np.linalg.inv(R).T
    z1, z2 = np.meshgrid(_GH_X, _GH_X, indexing="ij")
    w = np.outer(_GH_W, _GH_W)
    # u = mu + R^{-T} z
    x1 = mu[0] + Rinv_T[0, 0] * z1 + Rinv_T[0, 1] * z2
    x2 = mu[1] + Rinv_T[1, 0] * z1 + Rinv_T[1, 1] * z2
    f = (x1 - A) ** i * (x1 - B) ** j * (x2 - C) ** k * (x2 - D) ** l
    return np.exp(c0) / np.prod(np.diag(R)) * np.sum(w * f)


def eri_monomial(ijk_a, ijk_b, ijk_c, ijk_d, a, b, c, d, A, B, C, D, omega=None):
    """(ab|cd) of unnormalised monomial Gaussians x^i y^j z^k e^{-a r^2}.
    With omega, the operator is erf(omega r)/r = (2/sqrt(pi)) int_0^omega
    exp(-t^2 r^2) dt: the same integrand over t in [0, omega] (Gauss-Legendre
    on the finite interval)."""
    p, q = a + b, c + d
    rho = p * q / (p + q)
    total = 0.0
    for u, wu in zip(_GL_U, _GL_WU):
        if omega is None:
            t = np.sqrt(rho) * u / np.sqrt(1.0 - u * u)
            dt = np.sqrt(rho) * (1.0 - u * u) ** -1.5
        else:
            t, dt = omega * u, omega
        prod = 1.0
        for ax in range(3):
            prod *= _axis_integral(ijk_a[ax], ijk_b[ax], ijk_c[ax], ijk_d[ax],
                                   a, b, c, d, A[ax], B[ax], C[ax], D[ax], t)
        total += wu * dt * prod
    return 2.0 / np.sqrt(np.pi) * total


def _axis_potential(i, j, a, b, A, B, C, t):
    """int (x-A)^i (x-B)^j e^{-a(x-A)^2 - b(x-B)^2 - t^2 (x-C)^2} dx, exact by
    Gauss-Hermite after completing the square."""
    e = a + b + t * t
    m = (a * A + b * B + t * t * C) / e
    c0 = -(a * A * A + b * B * B + t * t * C * C) + e * m * m
    x = m + _GH_X / np.sqrt(e)
    f = (x - A) ** i * (x - B) ** j
    return np.exp(c0) / np.sqrt(e) * np.sum(_GH_W * f)


def potential_monomial(ijk_a, ijk_b, a, b, A, B, C):
    """int x^i.. e^{-a r_A^2} x^j.. e^{-b r_B^2} / |r - C| dr of unnormalised
    monomial Gaussians, by the Gaussian transform of 1/r; the t integral is
    mapped to u in [0, 1) by t = sqrt(p) u / sqrt(1 - u^2)."""
    p = a + b
    total = 0.0
    for u, wu in zip(_GL_U, _GL_WU):
        t = np.sqrt(p) * u / np.sqrt(1.0 - u * u)
        dt = np.sqrt(p) * (1.0 - u * u) ** -1.5
        prod = 1.0
        for ax in range(3):
            prod *= _axis_potential(ijk_a[ax], ijk_b[ax], a, b, A[ax], B[ax], C[ax], t)
        total += wu * dt * prod
    return 2.0 / np.sqrt(np.pi) * total


def _axis_st(i, j, a, b, A, B):
    """One-direction overlap int f_a f_b and derivative product
    int f_a' f_b' of f_a = (x-A)^i e^{-a(x-A)^2}, f_b = (x-B)^j e^{-b(x-B)^2},
    with the derivatives written out as polynomials, by Gauss-Hermite
    quadrature about the product centre."""
    p = a + b
    P = (a * A + b * B) / p
    c0 = -a * b / p * (A - B) ** 2
    x = P + _GH_X / np.sqrt(p)
    fa, fb = (x - A) ** i, (x - B) ** j
    dfa = (i * (x - A) ** (i - 1) if i > 0 else 0.0) - 2.0 * a * (x - A) ** (i + 1)
    dfb = (j * (x - B) ** (j - 1) if j > 0 else 0.0) - 2.0 * b * (x - B) ** (j + 1)
    f = np.exp(c0) / np.sqrt(p)
    return f * np.sum(_GH_W * fa * fb), f * np.sum(_GH_W * dfa * dfb)


def overlap_kinetic_monomial(ijk_a, ijk_b, a, b, A, B):
    """S = int a b and T = -1/2 int a lap(b) = 1/2 int grad(a).grad(b) of
    unnormalised monomial Gaussians (integration by parts; no recurrence)."""
    s, d = zip(*[_axis_st(ijk_a[k], ijk_b[k], a, b, A[k], B[k]) for k in range(3)])
    S = s[0] * s[1] * s[2]
    T = 0.5 * (d[0] * s[1] * s[2] + s[0] * d[1] * s[2] + s[0] * s[1] * d[2])
    return S, T
