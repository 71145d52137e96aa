"""Iteration logic of the SCF driver (paper_2406_14920_amd.scf) on the CPU:
the driver's algebra -- Fock matrix, energy, canonical orthogonalisation,
Pulay extrapolation, incremental J/K sums and the dynamic-precision schedule
-- run with a backend that returns the oracle's integrals, against the
oracle's own closed-shell SCF.  (The GPU precision and screening themselves
are covered by the GPU tests.)"""
import numpy as np
import pytest
import torch

import oracle
from paper_2406_14920_amd import scf, synth


class OracleBackend:
    def __init__(self, mol, nuclei):
        self.mol = mol
        self.B = oracle.OBasis(mol)
        self.nuclei = nuclei
        self.calls = []

    def one_electron(self):
        S, T = oracle.st(self.mol, basis_obj=self.B)
        V = oracle.vmatrix(self.mol, self.nuclei, basis_obj=self.B)
        return torch.tensor(S), torch.tensor(T + V)

    def jk_build(self, P):
        J, K = oracle.jk(self.mol, P=P.numpy(), basis_obj=self.B, tau=0.0, tau_prim=0.0)
        return torch.tensor(J), torch.tensor(K)

    def set_precision(self, name, tau):
        self.calls.append(("precision", name, tau))

    def set_density_screen(self, tau):
        self.calls.append(("screen", tau))

    def sync(self):
        pass


def _system():
    mol = synth.small_cluster(3, seed=12, tau=0.0, shellset=((0, 3), (0, 1), (1, 2), (1, 1), (2, 1)))
    nuc = np.concatenate([mol.xyz, -np.array([[3.0], [2.0], [3.0]])], axis=1)
    return mol, nuc, 4


def test_fp64_driver_matches_oracle_scf():
    mol, nuc, nocc = _system()
    ref, _, _ = oracle.rhf(mol, nuc, nocc, tau=0.0, tau_prim=0.0)
    res = scf.rhf(OracleBackend(mol, nuc), nuc, nocc, mode="fp64")
    assert res.converged
    assert res.energy == pytest.approx(ref, abs=1e-9)
    assert all(it.precision == "fp64" and not it.incremental for it in res.iterations)


def test_dynamic_driver_incremental_sums_and_schedule():
    """With exact integrals the incremental sums J(P) = J(P0) + sum J(dP)
    reproduce the same fixed point; the schedule starts in mixed precision
    with a threshold that follows the orbital gradient, rebuilds in full every
    rebuild_every iterations, and ends in double precision."""
    mol, nuc, nocc = _system()
    ref, _, _ = oracle.rhf(mol, nuc, nocc, tau=0.0, tau_prim=0.0)
    be = OracleBackend(mol, nuc)
    res = scf.rhf(be, nuc, nocc, mode="dynamic", rebuild_every=3, fp64_below=1e-4)
    assert res.converged
    assert res.energy == pytest.approx(ref, abs=1e-9)
    its = res.iterations
    assert its[0].precision == "mixed_all" and not its[0].incremental
    assert its[-1].precision == "fp64"
    first64 = next(i for i, it in enumerate(its) if it.precision == "fp64")
    assert not its[first64].incremental           # the switch is a full build
    run = 0
    for it in its:                                # at most rebuild_every incremental in a row
        run = run + 1 if it.incremental else 0
        assert run <= 3
    taus = [it.tau_mix for it in its if it.precision == "mixed_all"]
    assert all(1e-9 <= t <= 1e-3 for t in taus)
    screens = [c[1] for c in be.calls if c[0] == "screen"]
    assert screens[-1] == 0.0                     # left off afterwards
    assert any(s > 0.0 for s in screens)


def test_nuclear_repulsion():
    nuc = np.array([[0.0, 0.0, 0.0, 2.0], [0.0, 0.0, 2.0, 3.0], [1.0, 0.0, 0.0, -1.0]])
    ref = 2 * 3 / 2.0 + 2 * -1 / 1.0 + 3 * -1 / np.sqrt(5.0)
    assert scf.nuclear_repulsion(nuc) == pytest.approx(ref, rel=1e-15)
