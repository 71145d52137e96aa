"""GPU J, K, energy and gradient with the long-range operator erf(omega r)/r
(eqs. eri_longrange_definition, eri_longrange_formula) against the CPU
oracle, through the C ABI.

Bar: as for 1/r -- FP64 J, K within 1e-10 max|X|, gradient within
1e-10 max|g| + 1e-12 with a zero sum; mixed precision within 1e-6 absolute.
Screening uses the 1/r bounds on both sides.
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


def _micro():
    xyz = [[0.0, 0.0, 0.0], [1.2, 0.3, -0.4], [-0.5, 1.1, 0.8]]
    specs = [(0, 0, 3), (1, 0, 1), (2, 1, 2), (0, 1, 3), (1, 2, 1), (2, 2, 2), (0, 3, 1), (1, 3, 1),
             (2, 0, 2), (0, 2, 1)]
    return synth.custom(xyz, specs, seed=5, tau=0.0, exp_range=(0.15, 6.0), name="micro")


def _gpu(mol, omega, tau=None, tau_prim=None, precision="fp64"):
    torch = _torch()
    from paper_2406_14920_amd import JK
    jk = JK.from_molecule(mol, schwarz_thresh=mol.tau_schwarz if tau is None else tau, prim_thresh=tau_prim,
                          omega=omega, precision=precision)
    P = torch.tensor(mol.P, dtype=torch.float64, device="cuda")
    J, K = jk.jk(P)
    out = J.cpu().numpy(), K.cpu().numpy()
    jk.close()
    return out


def _check(X, Xr, tag, rtol=RTOL):
    err = np.abs(X - Xr).max()
    scale = np.abs(Xr).max()
    print("  %s: max|d| = %.3e  max|ref| = %.3e" % (tag, err, scale), flush=True)
    assert err <= rtol * scale, (tag, err, scale)


@pytest.mark.parametrize("omega", [0.2, 0.9, 4.0])
def test_micro_every_class_vs_oracle(omega):
    mol = _micro()
    print("case micro omega=%g" % omega, flush=True)
    J, K = _gpu(mol, omega, tau=0.0, tau_prim=0.0)
    Jr, Kr = oracle.jk(mol, tau=0.0, tau_prim=0.0, omega=omega)
    _check(J, Jr, "J")
    _check(K, Kr, "K")


def test_cluster_default_screening_vs_oracle():
    mol = synth.small_cluster(3, 2, tau=1e-11, name="c3")
    J, K = _gpu(mol, 0.4)
    Jr, Kr = oracle.jk(mol, omega=0.4)
    _check(J, Jr, "c3 J")
    _check(K, Kr, "c3 K")


def test_switching_operator_on_one_context():
    torch = _torch()
    from paper_2406_14920_amd import JK
    mol = synth.mol4()
    jk = JK.from_molecule(mol)
    P = torch.tensor(mol.P, dtype=torch.float64, device="cuda")
    J0, K0 = (t.cpu().numpy() for t in jk.jk(P))
    jk.set_omega(0.33)
    Jw, Kw = (t.cpu().numpy() for t in jk.jk(P))
    jk.set_omega(0.0)
    J1, K1 = (t.cpu().numpy() for t in jk.jk(P))
    jk.close()
    Jr, Kr = oracle.jk(mol, omega=0.33)
    _check(Jw, Jr, "mol4 omega J")
    _check(Kw, Kr, "mol4 omega K")
    _check(J1, J0, "back to 1/r J", 1e-13)
    _check(K1, K0, "back to 1/r K", 1e-13)


def test_gradient_vs_oracle():
    torch = _torch()
    from paper_2406_14920_amd import JK
    mol = _micro()
    jk = JK.from_molecule(mol, schwarz_thresh=0.0, prim_thresh=0.0, omega=0.7)
    P = torch.tensor(mol.P, dtype=torch.float64, device="cuda")
    g = jk.grad(P).cpu().numpy()
    jk.close()
    gr = oracle.grad(mol, tau=0.0, tau_prim=0.0, omega=0.7)
    err = np.abs(g - gr).max()
    print("  grad omega 0.7: max|dg| = %.3e  max|g| = %.3e" % (err, np.abs(gr).max()), flush=True)
    assert err <= RTOL * np.abs(gr).max() + 1e-12
    assert np.abs(g.sum(0)).max() <= 1e-9


@pytest.mark.parametrize("precision", ["mixed", "mixed_all"])
def test_mixed_vs_oracle(precision):
    mol = synth.mol4()
    J, K = _gpu(mol, 0.5, precision=precision)
    Jr, Kr = oracle.jk(mol, omega=0.5)
    for X, Xr, tag in ((J, Jr, "J"), (K, Kr, "K")):
        err = np.abs(X - Xr).max()
        print("  %s %s: max|d| = %.3e" % (precision, tag, err), flush=True)
        assert err <= 1e-6
