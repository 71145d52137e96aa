"""GPU batches of many molecules and the launch-shape autotuner: every
molecule's J and K from a batch must equal its own
build_jk (same kernels; only the order of floating-point atomic additions
may differ, so the bar is 1e-13 relative), on every replay, with the
program's own eager work and synchronisations between replays; the
autotuner must leave results unchanged to the same bar.  The stand-alone
builds are themselves held to the oracle by the parity tests.
"""
import numpy as np
import pytest

from paper_2406_14920_amd import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-13


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def _mols(n):
    # uneven sizes: the first molecules of the 64-molecule batch workload
    return synth.batch64()[:n]


def _close(X, Xr, tag):
    err = float((X - Xr).abs().max())
    scale = float(Xr.abs().max())
    assert err <= RTOL * scale, (tag, err, scale)


GRAPH_SKIP = ("batch graph recording is switched off: the recorded batch ended in a host-side segmentation "
              "fault inside eri_batch_build_jk on the MI355X runtime (twice, also without the per-context stream "
              "fork inside the recording) and the cause is not yet shown; kept for when it is re-enabled")


@pytest.mark.skip(reason=GRAPH_SKIP)
def test_batch_replays_match_standalone():
    torch = _torch()
    from paper_2406_14920_amd import JK, Batch
    mols = _mols(6)
    print("  sizes:", [m.nbf for m in mols], flush=True)
    jks = [JK.from_molecule(m) for m in mols]
    Ps = [torch.tensor(m.P, dtype=torch.float64, device="cuda") for m in mols]
    ref = [jk.jk(P) for jk, P in zip(jks, Ps)]
    torch.cuda.synchronize()
    b = Batch(jks)
    for rep in range(3):
        J, K = b.jk(Ps)
        torch.cuda.synchronize()
        for i in range(len(mols)):
            _close(J[i], ref[i][0], "J rep %d mol %d" % (rep, i))
            _close(K[i], ref[i][1], "K rep %d mol %d" % (rep, i))
        # eager work of the program between replays
        junk = torch.randn(512, 512, device="cuda", dtype=torch.float64)
        (junk @ junk).sum().item()
        for t in J + K:
            t.zero_()
        torch.cuda.synchronize()
    b.close()
    for jk in jks:
        jk.close()


@pytest.mark.skip(reason=GRAPH_SKIP)
def test_batch_rerecords_on_change():
    torch = _torch()
    from paper_2406_14920_amd import JK, Batch
    mols = _mols(3)
    jks = [JK.from_molecule(m) for m in mols]
    jks[1].set_precision("mixed")
    Ps = [torch.tensor(m.P, dtype=torch.float64, device="cuda") for m in mols]
    b = Batch(jks)
    J, K = b.jk(Ps)
    torch.cuda.synchronize()
    for i, (jk, P) in enumerate(zip(jks, Ps)):
        Jr, Kr = jk.jk(P)
        torch.cuda.synchronize()
        _close(J[i], Jr, "J mixed member %d" % i)
        _close(K[i], Kr, "K mixed member %d" % i)
    # new density tensors (new pointers) and a moved molecule
    Ps2 = [(P * 0.5).contiguous() for P in Ps]
    xyz = np.asarray(mols[2].xyz) + np.array([0.0, 0.1, -0.05])
    jks[2].set_geometry(xyz)
    J, K = b.jk(Ps2)
    torch.cuda.synchronize()
    for i, (jk, P) in enumerate(zip(jks, Ps2)):
        Jr, Kr = jk.jk(P)
        torch.cuda.synchronize()
        _close(J[i], Jr, "J after change %d" % i)
        _close(K[i], Kr, "K after change %d" % i)
    b.close()
    for jk in jks:
        jk.close()


def test_batch_direct_launches_match_standalone():
    """Streams mode: every molecule's build launched on one of the batch's
    streams, joined back; repeated calls with eager work between."""
    torch = _torch()
    from paper_2406_14920_amd import JK, Batch
    mols = _mols(6)
    print("  sizes:", [m.nbf for m in mols], flush=True)
    jks = [JK.from_molecule(m) for m in mols]
    jks[2].set_precision("mixed")
    Ps = [torch.tensor(m.P, dtype=torch.float64, device="cuda") for m in mols]
    ref = [tuple(t.clone() for t in jk.jk(P)) for jk, P in zip(jks, Ps)]
    torch.cuda.synchronize()
    b = Batch(jks, mode="streams")
    for rep in range(2):
        J, K = b.jk(Ps)
        torch.cuda.synchronize()
        for i in range(len(mols)):
            _close(J[i], ref[i][0], "J rep %d mol %d" % (rep, i))
            _close(K[i], ref[i][1], "K rep %d mol %d" % (rep, i))
        junk = torch.randn(256, 256, device="cuda", dtype=torch.float64)
        (junk @ junk).sum().item()
    b.close()
    for jk in jks:
        jk.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_all"])
def test_autotune_keeps_results(precision):
    torch = _torch()
    from paper_2406_14920_amd import JK
    mol = synth.small_cluster(5, 11, tau=1e-11, name="c5")
    jk = JK.from_molecule(mol, precision=precision)
    P = torch.tensor(mol.P, dtype=torch.float64, device="cuda")
    J0, K0 = jk.jk(P)
    J0, K0 = J0.clone(), K0.clone()
    tun = jk.autotune(P, reps=1)
    assert set(tun["kchunk"]) <= {8, 16, 32, 64, 128, 256, 512, 1024}
    assert set(tun["kcap"]) <= {0, 1024, 4096, 16384, 32768, 131072}
    J1, K1 = jk.jk(P)
    torch.cuda.synchronize()
    if precision != "fp64":
        # the tuner may move launches between the FP32 share and FP64, and a
        # change of ket grouping changes which quartets share a precision
        # tile: both results are mixed results, held to the mixed bar
        assert float((J1 - J0).abs().max()) <= 1e-6 and float((K1 - K0).abs().max()) <= 1e-6
    else:
        _close(J1, J0, "J after autotune")
        _close(K1, K0, "K after autotune")
    jk.close()


def test_batch_on_default_stream_is_ordered():
    """A batch created on the default stream (handle 0) forks from and joins
    back into that stream: densities produced by asynchronous work queued
    just before the call, and reads of J/K queued just after it, need no
    device-wide synchronisation."""
    torch = _torch()
    from paper_2406_14920_amd import JK, Batch
    mols = _mols(4)
    jks = [JK.from_molecule(m) for m in mols]
    Ps_host = [torch.tensor(m.P, dtype=torch.float64) for m in mols]
    ref = []
    for jk, Ph in zip(jks, Ps_host):
        J, K = jk.jk(Ph.cuda())
        ref.append((J.cpu(), K.cpu()))
    torch.cuda.synchronize()
    b = Batch(jks, stream=torch.cuda.default_stream())
    assert int(b.stream.cuda_stream) == 0
    with torch.cuda.stream(torch.cuda.default_stream()):
        for rep in range(2):
            # the densities come out of a long asynchronous chain on the default stream
            Ps = []
            for Ph in Ps_host:
                X = Ph.to("cuda", non_blocking=False) * 3.0
                for _ in range(20):
                    X = X * 0.5 + X * 0.5
                Ps.append((X / 3.0).contiguous())
            J, K = b.jk(Ps)
            got = [(j.cpu(), k.cpu()) for j, k in zip(J, K)]  # ordered reads, no synchronize
            for i in range(len(mols)):
                _close(got[i][0], ref[i][0], "J rep %d mol %d" % (rep, i))
                _close(got[i][1], ref[i][1], "K rep %d mol %d" % (rep, i))
    b.close()
    for jk in jks:
        jk.close()


def test_autotune_cache_roundtrip(tmp_path):
    """A tuning saved to the JSON cache is applied to a fresh context of the
    same workload without timing, and gives the same launch shapes and the
    same J, K (to the atomic-order bar)."""
    torch = _torch()
    from paper_2406_14920_amd import JK
    mol = synth.small_cluster(5, 11, tau=1e-11, name="c5")
    cache = str(tmp_path / "tuning.json")
    jk1 = JK.from_molecule(mol)
    P = torch.tensor(mol.P, dtype=torch.float64, device="cuda")
    t1 = jk1.autotune(P, reps=1, cache=cache, key="c5")
    J1, K1 = jk1.jk(P)
    jk2 = JK.from_molecule(mol)
    t2 = jk2.autotune(P, reps=1, cache=cache, key="c5")
    assert t1 == t2
    J2, K2 = jk2.jk(P)
    torch.cuda.synchronize()
    _close(J2, J1, "J after cached tuning")
    _close(K2, K1, "K after cached tuning")
    import json
    store = json.load(open(cache))
    assert "c5/fp64" in store and store["c5/fp64"]["exchange"]
    jk1.close()
    jk2.close()


def test_batch_latency_per_molecule():
    """Per-molecule completion times of a batch call: one per molecule,
    positive, none after the call's end (measured on the host around it)."""
    import time
    torch = _torch()
    from paper_2406_14920_amd import JK, Batch
    mols = [synth.small_cluster(n, 100 + n) for n in (2, 5, 3, 6)]
    jks = [JK.from_molecule(m) for m in mols]
    Ps = [torch.tensor(m.P, dtype=torch.float64, device="cuda") for m in mols]
    b = Batch(jks)
    b.jk(Ps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.jk(Ps)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    lat = b.latency()
    assert len(lat) == len(mols)
    assert all(0.0 < v <= wall_ms + 1.0 for v in lat), (lat, wall_ms)
    for jk, P, J, K in zip(jks, Ps, b.J, b.K):
        J0, K0 = jk.jk(P)
        _close(J, J0, "J batch")
        _close(K, K0, "K batch")
    b.close()


def test_batch_queue_launches_match_standalone():
    """Queue mode (the default for double-precision batches): one
    launch per kernel for all molecules.  Every molecule's J and K equal its
    own build_jk on repeated calls with eager work between; the plan is
    remade after a context changes (a moved molecule, a density screen)."""
    torch = _torch()
    from paper_2406_14920_amd import JK, Batch
    xyz = [[0.0, 0.0, 0.0], [1.9, 0.4, -0.3], [-0.7, 1.6, 0.9]]
    specs = [(0, 0, 3), (0, 0, 1), (0, 1, 2), (0, 2, 1), (0, 3, 1),
             (1, 0, 2), (1, 1, 1), (1, 3, 2),
             (2, 0, 1), (2, 2, 2), (2, 3, 1)]
    fshell = synth.custom(xyz, specs, seed=11, tau=1e-12, exp_range=(0.08, 60.0), name="f3")
    mols = _mols(7) + [fshell]
    print("  sizes:", [m.nbf for m in mols], flush=True)
    jks = [JK.from_molecule(m) for m in mols]
    Ps = [torch.tensor(m.P, dtype=torch.float64, device="cuda") for m in mols]
    ref = [tuple(t.clone() for t in jk.jk(P)) for jk, P in zip(jks, Ps)]
    torch.cuda.synchronize()
    b = Batch(jks)
    assert b.mode == "queue"
    for rep in range(3):
        J, K = b.jk(Ps)
        torch.cuda.synchronize()
        for i in range(len(mols)):
            _close(J[i], ref[i][0], "J rep %d mol %d" % (rep, i))
            _close(K[i], ref[i][1], "K rep %d mol %d" % (rep, i))
        junk = torch.randn(256, 256, device="cuda", dtype=torch.float64)
        (junk @ junk).sum().item()
        for t in J + K:
            t.fill_(7.0)
    info = b.queue_info()
    print("  queue plan:", info, flush=True)
    assert 0 < info["launches"] <= 200 and info["items"] > 0
    lat = b.latency()
    assert len(lat) == len(mols) and all(x > 0.0 for x in lat)
    # a moved molecule and a density-weighted screen on another: new plan
    xyz = np.asarray(mols[1].xyz) + np.array([0.05, -0.1, 0.02])
    jks[1].set_geometry(xyz)
    jks[3].set_density_screen(1e-12)
    ref2 = [tuple(t.clone() for t in jk.jk(P)) for jk, P in zip(jks, Ps)]
    J, K = b.jk(Ps)
    torch.cuda.synchronize()
    for i in range(len(mols)):
        _close(J[i], ref2[i][0], "J after change mol %d" % i)
        _close(K[i], ref2[i][1], "K after change mol %d" % i)
    # the streams form on the same batch gives the same results
    b.set_mode("streams")
    J, K = b.jk(Ps)
    torch.cuda.synchronize()
    for i in range(len(mols)):
        _close(J[i], ref2[i][0], "J streams mol %d" % i)
        _close(K[i], ref2[i][1], "K streams mol %d" % i)
    with pytest.raises(ValueError):
        b.set_mode("fused")
    b.close()
    for jk in jks:
        jk.close()


def test_batch_queue_graph_replays():
    """A queue-mode batch build after the first is a chain of kernel launches
    on the batch stream: captured into a HIP graph (torch's capture on that
    stream) and replayed three times with eager work between, every replay
    equals the eager build and follows new densities written into the same
    tensors."""
    torch = _torch()
    from paper_2406_14920_amd import JK, Batch
    mols = _mols(5)
    jks = [JK.from_molecule(m) for m in mols]
    Ps = [torch.tensor(m.P, dtype=torch.float64, device="cuda") for m in mols]
    s = torch.cuda.Stream()
    b = Batch(jks, stream=s)
    with torch.cuda.stream(s):
        J, K = b.jk(Ps)
    torch.cuda.synchronize()
    eager = [(j.clone(), k.clone()) for j, k in zip(J, K)]
    print("  eager done", flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.jk(Ps)
    torch.cuda.synchronize()
    print("  captured", flush=True)
    for rep in range(3):
        for t in J + K:
            t.fill_(-3.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(mols)):
            _close(J[i], eager[i][0], "J replay %d mol %d" % (rep, i))
            _close(K[i], eager[i][1], "K replay %d mol %d" % (rep, i))
        junk = torch.randn(300, 300, device="cuda", dtype=torch.float64)
        (junk @ junk).sum().item()
        print("  replay %d ok" % rep, flush=True)
    # new densities in the same tensors: the replay follows them
    for P in Ps:
        P.mul_(0.5)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    for i in range(len(mols)):
        _close(J[i], 0.5 * eager[i][0], "J new density mol %d" % i)
        _close(K[i], 0.5 * eager[i][1], "K new density mol %d" % i)
    del g
    b.close()
    for jk in jks:
        jk.close()


@pytest.mark.parametrize("members", ["mixed", "mixed_all"])
def test_batch_queue_mixed_precision_members(members):
    """Queue mode with mixed-precision members: their double- and
    single-precision shares run as separate batch kernels, with the same
    precision tiles as their own build_jk, so each molecule's J and K equal
    its own build (atomic order only); a member switched back to FP64 remakes
    the plan."""
    torch = _torch()
    from paper_2406_14920_amd import JK, Batch
    mols = _mols(6)
    jks = [JK.from_molecule(m) for m in mols]
    for i in (1, 3, 4):
        jks[i].set_precision(members)
    Ps = [torch.tensor(m.P, dtype=torch.float64, device="cuda") for m in mols]
    ref = [tuple(t.clone() for t in jk.jk(P)) for jk, P in zip(jks, Ps)]
    torch.cuda.synchronize()
    b = Batch(jks)
    assert b.mode == "queue"
    for rep in range(2):
        J, K = b.jk(Ps)
        torch.cuda.synchronize()
        for i in range(len(mols)):
            _close(J[i], ref[i][0], "J rep %d mol %d" % (rep, i))
            _close(K[i], ref[i][1], "K rep %d mol %d" % (rep, i))
        junk = torch.randn(256, 256, device="cuda", dtype=torch.float64)
        (junk @ junk).sum().item()
    launches_mixed = b.queue_info()["launches"]
    jks[3].set_precision("fp64")
    ref3 = tuple(t.clone() for t in jks[3].jk(Ps[3]))
    J, K = b.jk(Ps)
    torch.cuda.synchronize()
    _close(J[3], ref3[0], "J after switch")
    _close(K[3], ref3[1], "K after switch")
    for i in (0, 1, 2, 4, 5):
        _close(J[i], ref[i][0], "J after switch mol %d" % i)
        _close(K[i], ref[i][1], "K after switch mol %d" % i)
    assert launches_mixed > 0 and b.queue_info()["launches"] > 0
    b.close()
    for jk in jks:
        jk.close()
