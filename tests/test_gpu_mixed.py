"""GPU mixed precision ("mixed": the single-precision share on the launches
where it pays; "mixed_all": on every launch): tiles whose density-weighted Schwarz bound
Q_ab Q_cd max|D| is below the threshold run their primitive integrals in
single precision; bounds, Boys values, digestion and accumulation stay double.

Bar: max |X_mixed - X_oracle| <= 1e-6 (absolute, hartree) for X in {J, K} at
the default threshold 1e-5.  The all-single-precision limit (threshold above
every bound) is checked against the oracle relative to max|X| at a bound
derived from single-precision rounding, so every single-precision kernel is
exercised on every angular class; the all-double limit (threshold 0) must
reproduce the double-precision build.
"""
import numpy as np
import pytest

import oracle
from paper_2406_14920_amd import synth

pytestmark = pytest.mark.gpu

ABS_TOL = 1e-6     # mixed vs exact, absolute
FP32_REL = 2e-5    # every primitive integral in single precision, relative to max|X|


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def _run(mol, precision, mixed_thresh=1e-5, tau=None, tau_prim=None):
    torch = _torch()
    from paper_2406_14920_amd import JK
    jk = JK.from_molecule(mol, schwarz_thresh=mol.tau_schwarz if tau is None else tau, prim_thresh=tau_prim,
                          precision=precision, mixed_thresh=mixed_thresh)
    P = torch.tensor(mol.P, dtype=torch.float64, device="cuda")
    J, K = jk.jk(P)
    torch.cuda.synchronize()
    st = jk.stats()
    out = J.cpu().numpy(), K.cpu().numpy(), st
    jk.close()
    return out


def _micro():
    xyz = [[0.0, 0.0, 0.0], [1.2, 0.3, -0.4], [-0.5, 1.1, 0.8]]
    specs = [(0, 0, 3), (1, 0, 1), (2, 1, 2), (0, 1, 3), (1, 2, 1), (2, 2, 2), (0, 3, 1), (1, 3, 1),
             (2, 0, 2), (0, 2, 1)]
    return synth.custom(xyz, specs, seed=5, tau=0.0, exp_range=(0.15, 6.0), name="micro")


def _report(tag, X, Xr):
    err = np.abs(X - Xr).max()
    print("  %s: max|d| = %.3e  max|ref| = %.3e" % (tag, err, np.abs(Xr).max()), flush=True)
    return err


@pytest.mark.parametrize("case", ["micro", "c3"])
def test_all_single_precision_every_class(case):
    mol = _micro() if case == "micro" else synth.small_cluster(3, 2, tau=1e-11, name="c3")
    tau = 0.0 if case == "micro" else None
    print("case %s all-FP32 nbf=%d" % (case, mol.nbf), flush=True)
    J, K, st = _run(mol, "mixed_all", mixed_thresh=1e300, tau=tau, tau_prim=0.0 if case == "micro" else None)
    assert st["n_quartets_fp32"] == st["n_quartets"]
    Jr, Kr = oracle.jk(mol, tau=0.0 if case == "micro" else mol.tau_schwarz,
                       tau_prim=0.0 if case == "micro" else None)
    assert _report("J", J, Jr) <= FP32_REL * np.abs(Jr).max()
    assert _report("K", K, Kr) <= FP32_REL * np.abs(Kr).max()
    assert np.abs(J - J.T).max() <= 1e-14 * np.abs(J).max() and np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()


@pytest.mark.parametrize("mode", ["mixed", "mixed_all"])
def test_threshold_zero_is_double(mode):
    mol = synth.small_cluster(3, 1, tau=1e-11, name="c3")
    J, K, st = _run(mol, mode, mixed_thresh=0.0)
    assert st["n_quartets_fp32"] == 0
    J64, K64, _ = _run(mol, "fp64")
    assert np.abs(J - J64).max() <= 1e-13 * np.abs(J64).max()
    assert np.abs(K - K64).max() <= 1e-13 * np.abs(K64).max()


@pytest.mark.parametrize("mode", ["mixed", "mixed_all"])
def test_mol4_default_threshold_vs_oracle(mode):
    mol = synth.mol4()
    J, K, st = _run(mol, mode)
    print("  fp32 quartets %d of %d" % (st["n_quartets_fp32"], st["n_quartets"]), flush=True)
    Jr, Kr = oracle.jk(mol)
    assert _report("J", J, Jr) <= ABS_TOL
    assert _report("K", K, Kr) <= ABS_TOL


@pytest.mark.parametrize("mode", ["mixed", "mixed_all"])
def test_mol40_default_threshold(mode):
    """Full 40-atom workload: whole matrices against the double-precision
    build (itself held to the oracle at 1e-10 relative by the parity tests),
    and sampled shell blocks against the oracle directly."""
    mol = synth.mol40()
    J, K, st = _run(mol, mode)
    frac = st["n_quartets_fp32"] / st["n_quartets"]
    print("  fp32 quartets %d of %d (%.3f)" % (st["n_quartets_fp32"], st["n_quartets"], frac), flush=True)
    assert 0.0 < frac < 1.0
    J64, K64, _ = _run(mol, "fp64")
    assert _report("J vs fp64", J, J64) <= ABS_TOL
    assert _report("K vs fp64", K, K64) <= ABS_TOL
    B = oracle.OBasis(mol)
    rng = np.random.default_rng(41)
    ls = np.array([s.l for s in mol.shells])
    picks = []
    for la, lb in [(3, 3), (2, 0), (1, 1), (0, 0)]:
        picks.append((int(rng.choice(np.where(ls == la)[0])), int(rng.choice(np.where(ls == lb)[0]))))
    Jb, Kb = oracle.jk_blocks(mol, picks, picks, basis_obj=B)
    for (a, b), jb, kb in zip(picks, Jb, Kb):
        ra = slice(B.ao_off[a], B.ao_off[a] + 2 * B.l[a] + 1)
        rb = slice(B.ao_off[b], B.ao_off[b] + 2 * B.l[b] + 1)
        ej, ek = np.abs(J[ra, rb] - jb).max(), np.abs(K[ra, rb] - kb).max()
        print("  block (%d,%d): dJ=%.2e dK=%.2e" % (a, b, ej, ek), flush=True)
        assert ej <= ABS_TOL and ek <= ABS_TOL
