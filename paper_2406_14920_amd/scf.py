"""Closed-shell SCF driven by the library's J/K builds, with the paper's
dynamic precision and incremental Fock builds.

The Fock matrix is F = T + V + J(P) - K(P)/2 for the total density
P = 2 C_occ C_occ^T (J and K by eqs. j_definition and k_definition; T by eq.
kinetic_formula; V of the nuclei, q = -Z, by eq. v1e_formula), solved in the
canonically orthogonalised basis with Pulay's commutator extrapolation.  All
matrices stay on the GPU; the integrals come from the library, the small
dense linear algebra from torch.

Two ways to run the iterations:

* ``mode="fp64"``: every iteration builds J(P), K(P) from scratch in double
  precision -- the reference.
* ``mode="dynamic"``: the scheme the paper mentions for TeraChem (section
  "Performance", "DFT Calculations": the mixed-precision threshold can be
  updated during the SCF).  The paper gives no schedule; the one used here:
  iteration n runs in mixed precision with tau_mix = clamp(ratio * e_{n-1},
  tau_min, tau_max), e the largest element of the orbital gradient F P S -
  S P F of the previous iteration, until e falls below ``fp64_below``; from
  then on every build is double precision.  Builds are incremental --
  J(P_n) = J(P_{n-1}) + J(P_n - P_{n-1}), K likewise -- with the library's
  density-weighted screen at ``tau_dens``, so the work shrinks with the
  density change; a full build replaces the sums every ``rebuild_every``
  iterations and whenever the precision switches to double, so the final
  Fock matrix carries no accumulated single-precision error.

``backend`` is anything with the methods of :class:`GPUBackend` (the tests
also drive the iteration logic with a CPU backend).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


class GPUBackend:
    """The library's integrals for one context (a :class:`JK`)."""

    def __init__(self, jk, nuclei):
        import torch
        self.jk = jk
        self.torch = torch
        self.nuclei = torch.tensor(np.ascontiguousarray(nuclei, dtype=np.float64), device="cuda")

    def zeros(self, n):
        return self.torch.zeros((n, n), dtype=self.torch.float64, device="cuda")

    def one_electron(self):
        S, T = self.jk.one_electron()
        return S, T + self.jk.potential(self.nuclei)

    def jk_build(self, P):
        return self.jk.jk(P)

    def set_precision(self, name: str, tau_mix: float):
        self.jk.set_precision(name, tau_mix)

    def set_density_screen(self, tau: float):
        self.jk.set_density_screen(tau)

    def sync(self):
        self.torch.cuda.synchronize()


@dataclass
class Iteration:
    energy: float
    error: float
    precision: str
    tau_mix: float
    incremental: bool
    build_ms: float


@dataclass
class SCFResult:
    energy: float
    converged: bool
    iterations: List[Iteration] = field(default_factory=list)
    P: Optional[object] = None

    @property
    def build_ms(self) -> float:
        return sum(it.build_ms for it in self.iterations)


def nuclear_repulsion(nuclei) -> float:
    c = np.asarray(nuclei, float).reshape(-1, 4)
    d = np.linalg.norm(c[:, None, :3] - c[None, :, :3], axis=-1)
    iu = np.triu_indices(c.shape[0], 1)
    return float(np.sum(c[iu[0], 3] * c[iu[1], 3] / d[iu]))


def rhf(backend, nuclei, nocc: int, mode: str = "fp64", conv: float = 1e-9, grad_conv: float = 1e-6,
        max_iter: int = 100, ratio: float = 1e-2, tau_min: float = 1e-9, tau_max: float = 1e-3,
        fp64_below: float = 1e-5, tau_dens: float = 1e-12, rebuild_every: int = 6, diis: int = 8,
        lindep: float = 1e-6, level_shift: float = 0.0) -> SCFResult:
    """Closed-shell SCF (see the module docstring); nuclei rows x, y, z, q
    with q = -Z (their repulsion uses the charges as given).  Overlap
    eigenvalues below lindep are dropped from the orthogonalised basis (near
    linear dependence would otherwise amplify rounding noise in the orbital
    gradient by 1/lindep).  level_shift
    raises the virtual orbitals of the extrapolated Fock matrix by that many
    hartree before it is diagonalised (F + shift (S - S P S / 2)), which damps
    oscillating iterations and leaves the converged solution unchanged."""
    import torch
    if mode not in ("fp64", "dynamic"):
        raise ValueError("mode must be 'fp64' or 'dynamic'")
    S, H = backend.one_electron()
    n = S.shape[0]
    s, U = torch.linalg.eigh(S)
    keep = s > lindep
    X = U[:, keep] / torch.sqrt(s[keep])
    enuc = nuclear_repulsion(nuclei)

    def density(F):
        _, C = torch.linalg.eigh(X.T @ F @ X)
        Co = X @ C[:, :nocc]
        return 2.0 * Co @ Co.T

    P = density(H)
    Pb = None                   # density the running J, K belong to
    J = K = None
    Fs, Es = [], []
    out = SCFResult(energy=float("nan"), converged=False)
    err_prev = float("inf")
    E_old = None
    since_full = 0
    in_fp64 = mode == "fp64"
    for it in range(max_iter):
        # precision and build kind of this iteration
        if mode == "dynamic" and not in_fp64 and err_prev < fp64_below:
            in_fp64 = True
            Pb = None           # switch: full double-precision build
        if in_fp64:
            prec, tau = "fp64", 0.0
        else:
            tau = float(min(tau_max, max(tau_min, ratio * err_prev)))
            prec = "mixed_all"
        incremental = mode == "dynamic" and Pb is not None and since_full < rebuild_every
        backend.set_precision(prec, tau if prec != "fp64" else 1e-5)
        backend.set_density_screen(tau_dens if incremental else 0.0)
        backend.sync()
        t0 = time.perf_counter()
        if incremental:
            dJ, dK = backend.jk_build(P - Pb)
            J, K = J + dJ, K + dK
            since_full += 1
        else:
            J, K = backend.jk_build(P)
            since_full = 0
        backend.sync()
        ms = (time.perf_counter() - t0) * 1e3
        Pb = P
        F = H + J - 0.5 * K
        E = 0.5 * float(torch.sum(P * (H + F))) + enuc
        e = X.T @ (F @ P @ S - S @ P @ F) @ X
        err = float(e.abs().max())
        out.iterations.append(Iteration(E, err, prec, tau, incremental, ms))
        if E_old is not None and abs(E - E_old) < conv and err < grad_conv and in_fp64:
            out.energy, out.converged, out.P = E, True, P
            break
        E_old = E
        err_prev = err
        Fs.append(F)
        Es.append(e)
        Fs, Es = Fs[-diis:], Es[-diis:]
        m = len(Fs)
        B = -torch.ones((m + 1, m + 1), dtype=torch.float64, device=F.device)
        B[m, m] = 0.0
        for i in range(m):
            for j in range(m):
                B[i, j] = torch.sum(Es[i] * Es[j])
        rhs = torch.zeros(m + 1, dtype=torch.float64, device=F.device)
        rhs[m] = -1.0
        c = torch.linalg.lstsq(B.cpu(), rhs.cpu().unsqueeze(1)).solution[:m, 0].to(F.device)
        Fx = sum(ci * Fi for ci, Fi in zip(c, Fs))
        if level_shift:
            Fx = Fx + level_shift * (S - 0.5 * S @ P @ S)
        P = density(Fx)
    else:
        out.energy = out.iterations[-1].energy if out.iterations else float("nan")
        out.P = P
    backend.set_density_screen(0.0)
    return out
