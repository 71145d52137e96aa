"""Oracle-side basis conventions (test infrastructure only).

Normalisation and the Cartesian -> real-solid-harmonic transformation used by
the CPU oracle.  Written independently of the GPU library's own tables.

Conventions (section "Cartesian Gaussian basis functions", eqs.
contracted_basis / primtive_basis: every constant is folded into one C per
primitive):
  * a primitive x^i y^j z^k exp(-a r^2) of a shell with l = i+j+k carries the
    normalisation of its x^l component,
        N(a, l) = (2a/pi)^{3/4} (4a)^{l/2} / sqrt((2l-1)!!);
  * the contracted shell is rescaled so that its x^l component has unit norm,
    using the overlap formula (eq. overlap_formula) for two primitives on one
    centre, S = (pi/p)^{3/2} (2l-1)!! / (2p)^l with p = a_i + a_j;
  * spherical functions are real regular solid harmonics, ordered
    m = -l..l (p kept as x, y, z), each rescaled to unit norm.  They are built
    from the general expansion of a real solid harmonic in Cartesian monomials
    (Helgaker, Jorgensen, Olsen, Molecular Electronic-Structure Theory,
    eqs. 6.4.47-6.4.50).
"""
from __future__ import annotations

from math import comb, factorial, pi, sqrt
from typing import Dict, List, Tuple

import numpy as np


def dfact(n: int) -> int:
    """(n)!! with (-1)!! = 0!! = 1."""
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def cart_list(l: int) -> List[Tuple[int, int, int]]:
    """Cartesian components in lexicographic order, x power descending."""
    out = []
    for i in range(l, -1, -1):
        for j in range(l - i, -1, -1):
            out.append((i, j, l - i - j))
    return out


def prim_norm(a: float, l: int) -> float:
    return (2 * a / pi) ** 0.75 * (4 * a) ** (l / 2) / sqrt(dfact(2 * l - 1))


def normalised_coefs(l: int, exps: np.ndarray, coefs: np.ndarray) -> np.ndarray:
    """Fully normalised contraction coefficients C_i = c_i N(a_i, l) / sqrt(S)."""
    exps = np.asarray(exps, float)
    c = np.asarray(coefs, float) * np.array([prim_norm(a, l) for a in exps])
    S = 0.0
    for i in range(exps.size):
        for j in range(exps.size):
            p = exps[i] + exps[j]
            S += c[i] * c[j] * (pi / p) ** 1.5 * dfact(2 * l - 1) / (2 * p) ** l
    return c / sqrt(S)


def _monomial_overlap(m1, m2) -> float:
    """<x^i y^j z^k | x^i' y^j' z^k'> on one centre, in units where the
    normalised x^l component has norm 1 (same l on both sides)."""
    l = sum(m1)
    v = 1.0
    for a, b in zip(m1, m2):
        s = a + b
        if s % 2:
            return 0.0
        v *= dfact(s - 1)
    return v / dfact(2 * l - 1)


def _solid_harmonic_poly(l: int, m: int) -> Dict[Tuple[int, int, int], float]:
    """Real regular solid harmonic S_lm as {monomial: coefficient}."""
    am = abs(m)
    vm = 0.0 if m >= 0 else 0.5
    N = 1.0 / (2 ** am * factorial(l)) * sqrt(
        2 * factorial(l + am) * factorial(l - am) / (2.0 if m == 0 else 1.0))
    poly: Dict[Tuple[int, int, int], float] = {}
    for t in range((l - am) // 2 + 1):
        for u in range(t + 1):
            # v runs over vm, vm+1, ..., up to floor(am/2 - vm) + vm
            vmax = int(np.floor(am / 2 - vm)) + vm
            v = vm
            while v <= vmax + 1e-9:
                two_v = int(round(2 * v))
                c = ((-1) ** int(round(t + v - vm)) * (0.25 ** t) * comb(l, t)
                     * comb(l - t, am + t) * comb(t, u) * comb(am, two_v))
                px = 2 * t + am - 2 * u - two_v
                py = 2 * u + two_v
                pz = l - 2 * t - am
                key = (px, py, pz)
                poly[key] = poly.get(key, 0.0) + N * c
                v += 1.0
    return poly


def sph_matrix(l: int) -> np.ndarray:
    """T_l, shape (2l+1, ncart(l)): phi_sph[m] = sum_c T[m, c] phi_cart[c],
    for Cartesian primitives all carrying the x^l normalisation."""
    if l == 0:
        return np.ones((1, 1))
    if l == 1:
        return np.eye(3)  # p kept in (x, y, z) order
    carts = cart_list(l)
    idx = {c: k for k, c in enumerate(carts)}
    T = np.zeros((2 * l + 1, len(carts)))
    for row, m in enumerate(range(-l, l + 1)):
        poly = _solid_harmonic_poly(l, m)
        for mono, c in poly.items():
            T[row, idx[mono]] += c
        # unit norm with respect to the monomial metric
        S = np.array([[_monomial_overlap(a, b) for b in carts] for a in carts])
        nrm = T[row] @ S @ T[row]
        T[row] /= sqrt(nrm)
    return T


def cart_metric(l: int) -> np.ndarray:
    carts = cart_list(l)
    return np.array([[_monomial_overlap(a, b) for b in carts] for a in carts])


SPH = {l: sph_matrix(l) for l in range(0, 5)}
