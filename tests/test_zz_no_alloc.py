"""The allocation-free build (build_jk_static, C ABI) against build_jk on the
same contexts: two calls in a row on one GPU, the second with a smaller
input, each within the batch bar (the kernels are shared; only the order of
floating-point atomic additions may differ, so 1e-13 relative); oversized
and non-FP64 contexts are rejected with their documented codes."""
import pytest

from paper_2406_14920_amd import abi, synth

pytestmark = pytest.mark.gpu

RTOL = 1e-13


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def _pair(mol):
    torch = _torch()
    from paper_2406_14920_amd import JK
    jk = JK.from_molecule(mol)
    P = torch.tensor(mol.P, dtype=torch.float64, device="cuda")
    Jr, Kr = (t.clone() for t in jk.jk(P))
    J = torch.full_like(P, float("nan"))
    K = torch.full_like(P, float("nan"))
    with torch.cuda.stream(jk.stream):
        abi.build_jk_static(jk.ctx, P, J, K)
    torch.cuda.synchronize()
    for X, Xr, tag in ((J, Jr, "J"), (K, Kr, "K")):
        err = float((X - Xr).abs().max())
        scale = float(Xr.abs().max())
        print("  %s nbf=%d %s: max|d| %.2e (scale %.2e)" % (mol.name, mol.nbf, tag, err, scale), flush=True)
        assert err <= RTOL * scale, (mol.name, tag, err, scale)
    jk.close()


def test_static_build_matches_build_jk_twice():
    print("case mol4 then c3 (smaller)", flush=True)
    _pair(synth.mol4())                                            # 80 functions
    _pair(synth.small_cluster(3, 1, tau=1e-11, name="c3"))         # 63 functions, second call


def test_static_build_rejects_oversized_and_mixed():
    torch = _torch()
    from paper_2406_14920_amd import JK
    mol = synth.tm62()  # 1336 functions: needs more than the static array
    jk = JK.from_molecule(mol)
    P = torch.zeros((jk.nbf, jk.nbf), dtype=torch.float64, device="cuda")
    with pytest.raises(abi.EriError) as e:
        abi.build_jk_static(jk.ctx, P, P, P)
    assert e.value.code == abi.ERI_EINVAL and "scratch" in str(e.value)
    jk.close()
    mol = synth.mol4()
    jk = JK.from_molecule(mol, precision="mixed")
    P = torch.tensor(mol.P, dtype=torch.float64, device="cuda")
    with pytest.raises(abi.EriError) as e:
        abi.build_jk_static(jk.ctx, P, P.clone(), P.clone())
    assert e.value.code == abi.ERI_ESTATE
    jk.close()
