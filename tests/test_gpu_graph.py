"""One context's allocation-free build (build_jk_static) captured into a HIP
graph through torch's graph capture on the context's own stream, replayed
several times with the program's own eager work and synchronisations in
between; every replay must equal the eager build (and follow a new density
written into the same buffer)."""
import numpy as np
import pytest

from paper_2406_14920_amd import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def test_static_build_graph_replays_match_eager():
    torch = _torch()
    from paper_2406_14920_amd import JK, abi
    mol = synth.small_cluster(6, seed=44)
    s = torch.cuda.Stream()
    jk = JK.from_molecule(mol, stream=s)
    P = torch.tensor(mol.P, dtype=torch.float64, device="cuda")
    J = torch.empty_like(P)
    K = torch.empty_like(P)
    with torch.cuda.stream(s):
        abi.build_jk_static(jk.ctx, P, J, K)
    s.synchronize()
    J0, K0 = J.clone(), K.clone()
    print("eager done", flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        abi.build_jk_static(jk.ctx, P, J, K)
    s.synchronize()
    print("captured", flush=True)
    rng = np.random.default_rng(1)
    P2n = rng.standard_normal(P.shape)
    P2 = torch.tensor(0.5 * (P2n + P2n.T), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(s):
        abi.build_jk_static(jk.ctx, P2, J, K)
    s.synchronize()
    J2, K2 = J.clone(), K.clone()
    for rep in range(3):
        J.fill_(1.0)
        K.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        assert float((J - J0).abs().max()) <= 1e-13 * float(J0.abs().max()), rep
        assert float((K - K0).abs().max()) <= 1e-13 * float(K0.abs().max()), rep
        X = torch.randn(256, 256, device="cuda") @ torch.randn(256, 256, device="cuda")  # eager work in between
        torch.cuda.synchronize()
        print("replay %d ok" % rep, flush=True)
    P.copy_(P2)
    g.replay()
    torch.cuda.synchronize()
    assert float((J - J2).abs().max()) <= 1e-13 * float(J2.abs().max())
    assert float((K - K2).abs().max()) <= 1e-13 * float(K2.abs().max())
    del X
