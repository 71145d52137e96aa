"""GPU parity: J and K from the HIP library (through the C ABI) against the
CPU oracle on the same seeded inputs.

Bar (FP64): max |X_gpu - X_oracle| <= 1e-10 * max |X_oracle| for X in {J, K},
element by element (whole matrices for small systems, sampled shell blocks
at the full 40-atom size).
"""
import numpy as np
import pytest

import oracle
from paper_2406_14920_amd import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-10


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def _gpu_jk(mol, tau=None, tau_prim=None, want_j=True, want_k=True, spherical=True):
    torch = _torch()
    from paper_2406_14920_amd import JK
    tau = mol.tau_schwarz if tau is None else tau
    jk = JK.from_molecule(mol, schwarz_thresh=tau, prim_thresh=tau_prim, spherical=spherical)
    P = torch.tensor(mol.P, dtype=torch.float64, device="cuda")
    J, K = jk.jk(P, want_j=want_j, want_k=want_k)
    torch.cuda.synchronize()
    out = (None if J is None else J.cpu().numpy(), None if K is None else K.cpu().numpy())
    st = jk.stats()
    jk.close()
    return out[0], out[1], st


def _check(X, Xref, what):
    err = np.abs(X - Xref).max()
    scale = np.abs(Xref).max()
    print("  %s: max|d| = %.3e  max|ref| = %.3e  rel = %.3e" % (what, err, scale, err / scale), flush=True)
    assert err <= RTOL * scale, (what, err, scale)


def _micro():
    xyz = [[0.0, 0.0, 0.0], [1.2, 0.3, -0.4], [-0.5, 1.1, 0.8]]
    specs = [(0, 0, 3), (1, 0, 1), (2, 1, 2), (0, 1, 3), (1, 2, 1), (2, 2, 2), (0, 3, 1), (1, 3, 1),
             (2, 0, 2), (0, 2, 1)]
    return synth.custom(xyz, specs, seed=5, tau=0.0, exp_range=(0.15, 6.0), name="micro")


@pytest.mark.parametrize("case", ["micro", "mol4"])
def test_full_matrices_vs_oracle(case):
    mol = _micro() if case == "micro" else synth.mol4()
    tau = 0.0 if case == "micro" else mol.tau_schwarz
    print("case %s nbf=%d tau=%g prim_tau=0" % (case, mol.nbf, tau), flush=True)
    J, K, st = _gpu_jk(mol, tau=tau, tau_prim=0.0)
    Jr, Kr = oracle.jk(mol, tau=tau, tau_prim=0.0)
    _check(J, Jr, case + " J")
    _check(K, Kr, case + " K")
    assert np.allclose(J, J.T, atol=0) and np.allclose(K, K.T, atol=0)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_small_clusters(seed):
    """Grown 3-atom clusters with the 40-atom workload's shell set (all 100
    angular classes, contracted s/p shells), default screening thresholds."""
    mol = synth.small_cluster(3, seed, tau=1e-11, name="c3")
    print("case c3 seed=%d nbf=%d" % (seed, mol.nbf), flush=True)
    J, K, _ = _gpu_jk(mol)
    Jr, Kr = oracle.jk(mol)
    _check(J, Jr, "J")
    _check(K, Kr, "K")


def test_j_only_and_k_only():
    mol = _micro()
    J, _, _ = _gpu_jk(mol, tau=0.0, tau_prim=0.0, want_k=False)
    _, K, _ = _gpu_jk(mol, tau=0.0, tau_prim=0.0, want_j=False)
    Jr, Kr = oracle.jk(mol, tau=0.0, tau_prim=0.0)
    _check(J, Jr, "J only")
    _check(K, Kr, "K only")


def test_heavy_contractions_vs_oracle():
    """A heavy centre (s8 s8 p6 p6 d5 d5 f1) and two light atoms: ket pairs of
    up to 64 primitive pairs, so the exchange kernels walk their ket
    primitive loops in several batches and stop inside a batch on the
    primitive screen; default screening."""
    xyz = [[0.0, 0.0, 0.0], [3.6, 0.4, -0.3], [-1.2, 3.4, 0.8]]
    specs = [(0, 0, 8), (0, 0, 8), (0, 1, 6), (0, 1, 6), (0, 2, 5), (0, 2, 5), (0, 3, 1),
             (1, 0, 6), (1, 0, 3), (1, 1, 3), (1, 2, 1), (1, 3, 1),
             (2, 0, 6), (2, 1, 3), (2, 2, 1), (2, 3, 1)]
    mol = synth.custom(xyz, specs, seed=11, tau=1e-12, exp_range=(0.08, 60.0), name="heavy3")
    print("case heavy3 nbf=%d" % mol.nbf, flush=True)
    J, K, _ = _gpu_jk(mol)
    Jr, Kr = oracle.jk(mol)
    _check(J, Jr, "heavy3 J")
    _check(K, Kr, "heavy3 K")


def test_edge_single_s_shell():
    mol = synth.custom([[0.0, 0.0, 0.0]], [(0, 0, 1)], seed=3, tau=0.0)
    J, K, _ = _gpu_jk(mol, tau=0.0, tau_prim=0.0)
    Jr, Kr = oracle.jk(mol, tau=0.0, tau_prim=0.0)
    _check(J, Jr, "J")
    _check(K, Kr, "K")


def test_edge_only_f_shells_far_apart():
    """Two f shells 30 bohr apart: most quartets screened, empty classes."""
    mol = synth.custom([[0.0, 0.0, 0.0], [0.0, 0.0, 30.0]], [(0, 3, 1), (1, 3, 1)], seed=4, tau=1e-11)
    J, K, st = _gpu_jk(mol, tau=1e-11)
    Jr, Kr = oracle.jk(mol, tau=1e-11)
    _check(J, Jr, "J")
    _check(K, Kr, "K")


def test_repeat_builds_agree():
    torch = _torch()
    from paper_2406_14920_amd import JK
    mol = synth.small_cluster(4, 9)
    jk = JK.from_molecule(mol)
    P = torch.tensor(mol.P, dtype=torch.float64, device="cuda")
    J1, K1 = jk.jk(P)
    J2, K2 = jk.jk(P)
    torch.cuda.synchronize()
    # FP64 atomics may reorder sums: agree to rounding
    assert torch.allclose(J1, J2, rtol=0, atol=1e-13 * float(J1.abs().max()))
    assert torch.allclose(K1, K2, rtol=0, atol=1e-13 * float(K1.abs().max()))
    jk.close()


def test_mol40_sampled_blocks():
    """40-atom workload at full size, default thresholds, sampled shell blocks."""
    mol = synth.mol40()
    print("case mol40 nbf=%d" % mol.nbf, flush=True)
    J, K, st = _gpu_jk(mol)
    print("  quartets %d pairs %d" % (st["n_quartets"], st["n_pairs"]), flush=True)
    B = oracle.OBasis(mol)
    rng = np.random.default_rng(40)
    ls = np.array([s.l for s in mol.shells])
    picks = []
    for la, lb in [(3, 3), (3, 0), (2, 1), (0, 0), (1, 1), (3, 2)]:
        a = int(rng.choice(np.where(ls == la)[0]))
        b = int(rng.choice(np.where(ls == lb)[0]))
        picks.append((a, b))
    Jb, Kb = oracle.jk_blocks(mol, picks, picks, basis_obj=B)
    scaleJ, scaleK = np.abs(J).max(), np.abs(K).max()
    for (a, b), jb, kb in zip(picks, Jb, Kb):
        ra = slice(B.ao_off[a], B.ao_off[a] + 2 * B.l[a] + 1)
        rb = slice(B.ao_off[b], B.ao_off[b] + 2 * B.l[b] + 1)
        ej = np.abs(J[ra, rb] - jb).max()
        ek = np.abs(K[ra, rb] - kb).max()
        print("  block (%d,%d) l=(%d,%d): dJ=%.2e dK=%.2e" % (a, b, B.l[a], B.l[b], ej, ek), flush=True)
        assert ej <= RTOL * scaleJ and ek <= RTOL * scaleK
