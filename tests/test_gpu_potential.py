"""GPU point-charge potential V and its gradient (eqs. v1e_definition,
v1e_summation_over_C, v1e_formula; SI eqs. si_v1e_derivative_A/B/C) against
the CPU oracle, through the C ABI.

Charges are the atoms' nuclei (q = -Z, sitting on basis-function centres,
so one-centre pairs meet T = 0) plus QM/MM-style embedding charges
(synth.point_charges).  Bar: V within 1e-10 max|V| element by element;
gradients within 1e-10 max|g| + 1e-12; double precision throughout, so the
only differences are summation order (terms of one sign per charge, a few
hundred at most per element) and the pairs that fail the Schwarz rule
(absent on both sides only when the threshold is 0).
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


def _charges(mol, n_mm, seed):
    parts = [synth.nuclei(mol, seed)]
    if n_mm:
        parts.append(synth.point_charges(mol, n_mm, seed=seed + 1))
    return np.ascontiguousarray(np.concatenate(parts, axis=0))


def _gpu(mol, chg, tau=None, grad=True):
    torch = _torch()
    from paper_2406_14920_amd import JK
    jk = JK.from_molecule(mol, schwarz_thresh=mol.tau_schwarz if tau is None else tau)
    c = torch.tensor(chg, dtype=torch.float64, device="cuda")
    V = jk.potential(c)
    out = {"V": V.cpu().numpy()}
    if grad:
        P = torch.tensor(0.5 * (mol.P + mol.P.T), dtype=torch.float64, device="cuda")
        ga, gc = jk.potential_grad(c, P)
        out["ga"], out["gc"] = ga.cpu().numpy(), gc.cpu().numpy()
    return out, jk


def _close(name, got, ref, rtol=RTOL, atol=0.0):
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(got - ref).max() if ref.size else 0.0
    assert err <= rtol * scale + atol, "%s: max|d| %.3e vs scale %.3e" % (name, err, scale)


@pytest.mark.parametrize("case", ["micro", "mol4"])
def test_potential_and_gradient_vs_oracle(case):
    mol = _micro() if case == "micro" else synth.mol4()
    chg = _charges(mol, 12 if case == "micro" else 40, seed=3)
    print("case %s nbf %d charges %d" % (case, mol.nbf, chg.shape[0]), flush=True)
    got, _ = _gpu(mol, chg)
    Vr = oracle.vmatrix(mol, chg)
    _close("V", got["V"], Vr)
    assert np.array_equal(got["V"], got["V"].T) or np.abs(got["V"] - got["V"].T).max() <= 1e-14 * np.abs(Vr).max()
    P = 0.5 * (mol.P + mol.P.T)
    ga, gc = oracle.vgrad(mol, chg, P=P)
    _close("gatom", got["ga"], ga, atol=1e-12)
    _close("gchg", got["gc"], gc, atol=1e-12)
    tot = got["ga"].sum(0) + got["gc"].sum(0)
    assert np.abs(tot).max() <= 1e-10 * max(1.0, np.abs(ga).max())


def test_cartesian_output():
    """A context with Cartesian output returns the symmetric Cartesian V
    (ncart per shell), one with spherical output the oracle's V."""
    torch = _torch()
    from paper_2406_14920_amd import JK
    mol = _micro()
    chg = _charges(mol, 5, seed=8)
    c = torch.tensor(chg, dtype=torch.float64, device="cuda")
    jk_s = JK.from_molecule(mol, schwarz_thresh=0.0)
    jk_c = JK.from_molecule(mol, schwarz_thresh=0.0, spherical=False)
    Vs = jk_s.potential(c).cpu().numpy()
    Vc = jk_c.potential(c).cpu().numpy()
    assert Vc.shape[0] > Vs.shape[0]
    assert np.abs(Vc - Vc.T).max() <= 1e-14 * np.abs(Vc).max()
    _close("V_sph", Vs, oracle.vmatrix(mol, chg))


def test_no_charges_and_repeat_calls():
    torch = _torch()
    mol = synth.mol4()
    chg = _charges(mol, 25, seed=4)
    got, jk = _gpu(mol, chg)
    c = torch.tensor(chg, dtype=torch.float64, device="cuda")
    P = torch.tensor(0.5 * (mol.P + mol.P.T), dtype=torch.float64, device="cuda")
    for _ in range(2):
        V = jk.potential(c).cpu().numpy()
        ga, gc = jk.potential_grad(c, P)
        assert np.array_equal(V, got["V"])
        assert np.array_equal(ga.cpu().numpy(), got["ga"])
        assert np.array_equal(gc.cpu().numpy(), got["gc"])
    empty = torch.zeros((0, 4), dtype=torch.float64, device="cuda")
    V0 = jk.potential(empty).cpu().numpy()
    ga0, gc0 = jk.potential_grad(empty, P)
    assert not V0.any() and not ga0.cpu().numpy().any() and gc0.shape == (0, 3)
    # a J/K build on the same context in between leaves V unchanged
    jk.jk(P)
    assert np.array_equal(jk.potential(c).cpu().numpy(), got["V"])


def test_mol40_nuclei_vs_oracle_and_embedding_linearity():
    """mol40 (840 spherical bf): V of the 40 nuclei against the oracle in
    full; with 2000 embedding charges (the size the benchmark times) V is
    linear in the charge set and the gradient sums to zero, and the charge
    rows of a few charges match the oracle run on those charges alone."""
    torch = _torch()
    from paper_2406_14920_amd import JK
    mol = synth.mol40()
    nuc = synth.nuclei(mol, seed=1)
    mm = synth.point_charges(mol, 2000, seed=2)
    jk = JK.from_molecule(mol)
    cn = torch.tensor(nuc, dtype=torch.float64, device="cuda")
    cm = torch.tensor(mm, dtype=torch.float64, device="cuda")
    call = torch.cat([cn, cm], 0).contiguous()
    print("mol40 nuclei", flush=True)
    Vn = jk.potential(cn).cpu().numpy()
    _close("V nuclei", Vn, oracle.vmatrix(mol, nuc))
    print("mol40 embedding", flush=True)
    Vm = jk.potential(cm).cpu().numpy()
    Va = jk.potential(call).cpu().numpy()
    _close("V linear", Va, Vn + Vm, rtol=1e-12)
    P = torch.tensor(0.5 * (mol.P + mol.P.T), dtype=torch.float64, device="cuda")
    ga, gc = jk.potential_grad(call, P)
    ga, gc = ga.cpu().numpy(), gc.cpu().numpy()
    tot = ga.sum(0) + gc.sum(0)
    assert np.abs(tot).max() <= 1e-9 * max(1.0, np.abs(ga).max())
    pick = [3, 777, 1999]
    _, gcr = oracle.vgrad(mol, mm[pick], P=0.5 * (mol.P + mol.P.T))
    _close("gchg rows", gc[[40 + i for i in pick]], gcr, atol=1e-12)
