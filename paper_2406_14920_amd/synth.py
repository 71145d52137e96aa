"""Seeded synthetic molecules and densities for the J/K workloads.

This module only draws random numbers: atom positions, shell exponents, raw
contraction coefficients and a random orthonormal orbital block.  It holds
none of the integral arithmetic (no normalisation, no integrals, no screening),
so both the CPU oracle (through the tests) and the GPU library can take their
inputs from it without sharing any part of the method.

The paper's molecules (alkanes, taxol, metal complexes with cc-pVxZ/def2 bases,
section "Performance") are not available; these draws stand in for them with
the same ingredients: contracted Cartesian Gaussian shells up to f on atoms at
bonding distances (eq. contracted_basis / primtive_basis).

Workloads (exponent ranges and placement rules in the functions below):
  mol4    4 atoms in a 6 bohr cube, shells s3 s1 p3 p1 d1 f1            (80 sph)
  mol40   40-atom grown cluster, shells s6 s3 s1 p3 p1 d1 f1            (840 sph)
  tm62    2 heavy centres + 60 light atoms                              (1336 sph)
  mol20   20-atom grown cluster (gradient workload)                      (420 sph)
  batch64 64 grown clusters of 5..30 atoms (serving-style batch)
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

# (l, nprim) per shell
LIGHT4_SHELLS: Tuple[Tuple[int, int], ...] = ((0, 3), (0, 1), (1, 3), (1, 1), (2, 1), (3, 1))
LIGHT_SHELLS: Tuple[Tuple[int, int], ...] = ((0, 6), (0, 3), (0, 1), (1, 3), (1, 1), (2, 1), (3, 1))
HEAVY_SHELLS: Tuple[Tuple[int, int], ...] = (
    (0, 8), (0, 8), (0, 8), (1, 6), (1, 6), (2, 5), (2, 5), (2, 5), (3, 1), (3, 1))


@dataclass
class Shell:
    atom: int
    l: int
    exps: np.ndarray    # [nprim], descending
    coefs: np.ndarray   # [nprim], raw coefficients of normalised primitives


@dataclass
class Molecule:
    name: str
    xyz: np.ndarray                 # [natom, 3] bohr
    shells: List[Shell]
    P: np.ndarray                   # [nbf, nbf] symmetric density in the spherical AO basis
    nocc: int
    tau_schwarz: float
    meta: dict = field(default_factory=dict)

    @property
    def natom(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nbf(self) -> int:
        return int(sum(2 * s.l + 1 for s in self.shells))


def nsph(l: int) -> int:
    return 2 * l + 1


def _unit(rng: np.random.Generator) -> np.ndarray:
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


def _box_positions(rng, natom, box, min_sep):
    while True:
        x = rng.uniform(0.0, box, size=(natom, 3))
        d = np.linalg.norm(x[:, None, :] - x[None, :, :], axis=-1)
        d[np.diag_indices(natom)] = np.inf
        if d.min() >= min_sep:
            return x


def _grow_cluster(rng, natom, dmin=2.6, dmax=3.0, seed_xyz=None, heavy=0,
                  heavy_dmin=3.5, heavy_dmax=3.9):
    """Grow a cluster: each new atom is placed at distance U(dmin, dmax) from a
    randomly chosen existing atom in a random direction and accepted if it is at
    least dmin from every light atom and heavy_dmin from every heavy atom.
    The first `heavy` atoms of seed_xyz are heavy centres."""
    xyz = [np.zeros(3)] if seed_xyz is None else [np.asarray(p, float) for p in seed_xyz]
    while len(xyz) < natom:
        parent = int(rng.integers(len(xyz)))
        if parent < heavy:
            d = rng.uniform(heavy_dmin, heavy_dmax)
        else:
            d = rng.uniform(dmin, dmax)
        cand = xyz[parent] + d * _unit(rng)
        arr = np.asarray(xyz)
        dist = np.linalg.norm(arr - cand, axis=1)
        ok_heavy = bool(np.all(dist[:heavy] >= heavy_dmin)) if heavy else True
        ok_light = bool(np.all(dist[heavy:] >= dmin - 1e-12))
        if ok_heavy and ok_light:
            xyz.append(cand)
    return np.asarray(xyz)


def _draw_shells(rng, atoms_shellsets: Sequence[Tuple[Tuple[int, int], ...]],
                 ranges: Sequence[Tuple[float, float]]) -> List[Shell]:
    """Exponents log-uniform in the atom's range (sorted descending within a
    shell), then coefficients U(0.1, 1); exponents of all shells first."""
    exps_all = []
    for ia, (sset, (lo, hi)) in enumerate(zip(atoms_shellsets, ranges)):
        for (l, n) in sset:
            e = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))
            exps_all.append((ia, l, np.sort(e)[::-1].copy()))
    shells = []
    for (ia, l, e) in exps_all:
        c = rng.uniform(0.1, 1.0, size=e.size)
        shells.append(Shell(atom=ia, l=l, exps=e, coefs=c))
    return shells


def _density(rng, nbf: int, nocc: int) -> np.ndarray:
    """P = C C^T with C a random Euclidean-orthonormal nbf x nocc block."""
    a = rng.standard_normal((nbf, nocc))
    q, _ = np.linalg.qr(a)
    P = q @ q.T
    return 0.5 * (P + P.T)


def _finish(name, rng, xyz, shells, tau, nocc=None, meta=None) -> Molecule:
    nbf = int(sum(nsph(s.l) for s in shells))
    if nocc is None:
        nocc = max(1, int(round(nbf / 10)))
    P = _density(rng, nbf, nocc)
    return Molecule(name=name, xyz=xyz, shells=shells, P=P, nocc=nocc,
                    tau_schwarz=tau, meta=dict(meta or {}))


def mol4(seed: int = 14921) -> Molecule:
    rng = np.random.default_rng(seed)
    xyz = _box_positions(rng, 4, 6.0, 2.0)
    shells = _draw_shells(rng, [LIGHT4_SHELLS] * 4, [(0.1, 1e3)] * 4)
    return _finish("mol4", rng, xyz, shells, 1e-12, nocc=10)


def cluster(natom: int, seed, name: str = "cluster", tau: float = 1e-11,
            exp_range=(0.08, 5e3)) -> Molecule:
    rng = np.random.default_rng(seed)
    xyz = _grow_cluster(rng, natom)
    shells = _draw_shells(rng, [LIGHT_SHELLS] * natom, [exp_range] * natom)
    return _finish(name, rng, xyz, shells, tau)


def mol40(seed: int = 14922) -> Molecule:
    return cluster(40, seed, "mol40")


def tm62(seed: int = 14923) -> Molecule:
    rng = np.random.default_rng(seed)
    heavy = [np.array([-2.4, 0.0, 0.0]), np.array([2.4, 0.0, 0.0])]
    xyz = _grow_cluster(rng, 62, seed_xyz=heavy, heavy=2)
    sets = [HEAVY_SHELLS] * 2 + [LIGHT_SHELLS] * 60
    ranges = [(0.05, 2e5)] * 2 + [(0.08, 5e3)] * 60
    shells = _draw_shells(rng, sets, ranges)
    return _finish("tm62", rng, xyz, shells, 1e-11)


def mol20(seed: int = 14924) -> Molecule:
    return cluster(20, seed, "mol20")


def batch64(seed: int = 14925, n: int = 64, lo: int = 5, hi: int = 30) -> List[Molecule]:
    children = np.random.SeedSequence(seed).spawn(n)
    mols = []
    for i, ss in enumerate(children):
        rng = np.random.default_rng(ss)
        natom = int(rng.integers(lo, hi + 1))
        xyz = _grow_cluster(rng, natom)
        shells = _draw_shells(rng, [LIGHT_SHELLS] * natom, [(0.08, 5e3)] * natom)
        mols.append(_finish(f"batch64[{i}]", rng, xyz, shells, 1e-11))
    return mols


def small_cluster(natom: int, seed: int, shellset=LIGHT_SHELLS, exp_range=(0.08, 5e3),
                  tau: float = 1e-11, name: str = "small") -> Molecule:
    """A grown cluster with a chosen shell set (parity tests)."""
    rng = np.random.default_rng(seed)
    xyz = _grow_cluster(rng, natom)
    shells = _draw_shells(rng, [tuple(shellset)] * natom, [exp_range] * natom)
    return _finish(name, rng, xyz, shells, tau)


def custom(xyz, shell_specs, seed: int = 0, tau: float = 1e-12, nocc=None,
           exp_range=(0.1, 10.0), name: str = "custom") -> Molecule:
    """Molecule from explicit positions and (atom, l, nprim) shell specs; the
    exponents/coefficients/density are drawn from `seed`."""
    rng = np.random.default_rng(seed)
    xyz = np.asarray(xyz, float).reshape(-1, 3)
    exps_all = []
    for (ia, l, n) in shell_specs:
        e = np.exp(rng.uniform(np.log(exp_range[0]), np.log(exp_range[1]), size=n))
        exps_all.append((ia, l, np.sort(e)[::-1].copy()))
    shells = [Shell(atom=ia, l=l, exps=e, coefs=rng.uniform(0.1, 1.0, size=e.size))
              for (ia, l, e) in exps_all]
    nbf = int(sum(nsph(s.l) for s in shells))
    if nocc is None:
        nocc = max(1, nbf // 4)
    return _finish(name, rng, xyz, shells, tau, nocc=nocc)


WORKLOADS = {"mol4": mol4, "mol40": mol40, "tm62": tm62, "mol20": mol20}


def nuclei(mol: Molecule, seed: int = 0, even: bool = False) -> np.ndarray:
    """Nuclear point charges of the atoms, rows x, y, z, q with q = -Z and Z
    drawn from {1, 6, 7, 8} (the synthetic atoms carry no element); with
    even=True the first atom's Z moves by one where needed so that the
    electron count sum Z is even (closed shell)."""
    rng = np.random.default_rng(seed)
    Z = rng.choice(np.array([1.0, 6.0, 7.0, 8.0]), size=mol.natom)
    if even and int(Z.sum()) % 2:
        Z[0] += 1.0 if Z[0] in (1.0, 6.0) else -1.0
    return np.concatenate([mol.xyz, -Z[:, None]], axis=1)


def point_charges(mol: Molecule, n: int, seed: int = 0, rmin: float = 2.0, pad: float = 8.0) -> np.ndarray:
    """n embedding point charges (QM/MM style), rows x, y, z, q: uniform in the
    atoms' bounding box widened by `pad` bohr, none closer than `rmin` bohr to
    an atom, q uniform in [-1, 1]."""
    rng = np.random.default_rng(seed)
    lo = mol.xyz.min(axis=0) - pad
    hi = mol.xyz.max(axis=0) + pad
    out = np.zeros((0, 3))
    while out.shape[0] < n:
        x = rng.uniform(lo, hi, size=(max(64, 2 * (n - out.shape[0])), 3))
        d2 = ((x[:, None, :] - mol.xyz[None, :, :]) ** 2).sum(-1).min(axis=1)
        out = np.concatenate([out, x[d2 >= rmin * rmin]], axis=0)
    q = rng.uniform(-1.0, 1.0, size=n)
    return np.concatenate([out[:n], q[:, None]], axis=1)


def molecular_grid(mol: Molecule, nrad: int = 40, ntheta: int = 11, nphi: int = 22, rm: float = 1.0):
    """Atom-centred integration grid (the paper's molecular grids are not
    specified): per atom, nrad radial nodes of Gauss-Chebyshev quadrature of
    the second kind mapped by r = rm (1 + x) / (1 - x), times ntheta
    Gauss-Legendre nodes in cos(theta) and nphi equally spaced phi, with
    Becke's fuzzy-cell partition (three iterations of f(u) = 1.5u - 0.5u^3) for
    the weights.  Points come atom by atom and radial shell by radial shell,
    so neighbouring points lie close together.  Returns (points [n, 3],
    weights [n]).  Geometry only: no random numbers and none of the integral
    arithmetic."""
    k = np.arange(1, nrad + 1)
    x = np.cos(k * np.pi / (nrad + 1))
    wx = np.pi / (nrad + 1) * np.sin(k * np.pi / (nrad + 1)) ** 2 / np.sqrt(1.0 - x * x)
    r = rm * (1.0 + x) / (1.0 - x)
    wr = wx * 2.0 * rm / (1.0 - x) ** 2 * r * r
    ct, wt = np.polynomial.legendre.leggauss(ntheta)
    st = np.sqrt(1.0 - ct * ct)
    ph = 2.0 * np.pi * np.arange(nphi) / nphi
    dirs = np.stack([(st[:, None] * np.cos(ph)[None, :]).ravel(), (st[:, None] * np.sin(ph)[None, :]).ravel(),
                     np.repeat(ct, nphi)], axis=1)
    wa = np.repeat(wt, nphi) * (2.0 * np.pi / nphi)
    xyz = mol.xyz
    nat = mol.natom
    R = np.linalg.norm(xyz[:, None, :] - xyz[None, :, :], axis=-1) + np.eye(nat)
    pts, wts = [], []
    for a in range(nat):
        p = (xyz[a][None, None, :] + r[:, None, None] * dirs[None, :, :]).reshape(-1, 3)
        w = (wr[:, None] * wa[None, :]).ravel()
        d = np.linalg.norm(p[:, None, :] - xyz[None, :, :], axis=-1)      # [n, nat]
        cell = np.empty((p.shape[0], nat))
        for A in range(nat):
            s = (d[:, A:A + 1] - d) / R[A][None, :]                       # mu_AB, [n, B]
            for _ in range(3):
                s = s * (1.5 - 0.5 * s * s)
            s = 0.5 * (1.0 - s)
            s[:, A] = 1.0
            cell[:, A] = np.prod(s, axis=1)
        pts.append(p)
        wts.append(w * cell[:, a] / np.sum(cell, axis=1))
    return np.concatenate(pts, 0), np.concatenate(wts, 0)
