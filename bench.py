#!/usr/bin/env python3
"""Benchmark: one J+K build (one SCF iteration's Coulomb and exchange
matrices) of the 40-atom workload (840 spherical functions, shells
s6 s3 s1 p3 p1 d1 f1 per atom, Schwarz threshold 1e-11) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed]

Prints one JSON line.  value = contracted spherical ERIs represented per
second (sum over kept unique shell quartets of prod(2l+1), divided by the
J+K time); ms_per_step = the J+K build time.  Inputs (P) are resident in HBM
before the timed region; setup (pairs, Schwarz factors) is outside it.

The roofline entry is for the dominant kernel of the step: its algorithmic
FLOPs per launch (the library's fixed FLOP model per primitive quartet,
primitive quartets counted by the library with the kernels' own screening
loops) divided by its average launch
time, taken from HIP events that the library records on its launch stream
during a profiled pass of the same number of steps right after the timed
region (the library runs a profiled build on one stream, so each event pair
brackets one kernel; the timed region itself runs the concurrent path).  cpu_baseline times the CPU oracle on a bounded random
sample of the same workload's kept shell quartets.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6  # TFLOP/s: 256 CU x 4 SIMD x 16 FP64 lanes x 2 FLOP x 2.4 GHz
METRIC = "J+K build ms/iter + ERIs/s, FP32-mixed vs FP64 at ≤1e-6 max|ΔJ,ΔK|"


def _kernel_src_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2406_14920_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def _traffic(kernel_name: str, launches_per_step: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_mol40.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("src_hash") != _kernel_src_hash():
        return None
    row = d.get("kernels", {}).get(kernel_name)
    if not row:
        return None
    return row.get("bytes_per_launch")


def cpu_baseline(mol, target_s: float = 15.0):
    """Oracle rate on a random sample of the workload's kept shell quartets."""
    import oracle
    B = oracle.OBasis(mol)
    Q = B.schwarz()
    tau = mol.tau_schwarz
    tau_prim = 1e-2 * tau
    B.prim_bounds()
    n = B.nshell
    pairs = np.array([(a, b) for a in range(n) for b in range(a + 1)], np.int32)
    qp = Q[pairs[:, 0], pairs[:, 1]]
    rng = np.random.default_rng(2024)
    nsph = 2 * B.l + 1

    def draw(k):
        out, have = [], 0
        while have < k:
            i = rng.integers(len(pairs), size=4 * k)
            j = rng.integers(len(pairs), size=4 * k)
            ok = qp[i] * qp[j] >= tau
            blk = np.concatenate([pairs[i[ok]], pairs[j[ok]]], axis=1)
            out.append(blk)
            have += len(blk)
        return np.ascontiguousarray(np.concatenate(out)[:k], np.int32)

    q = draw(20000)  # pilot run sizes the sample to about target_s
    t = time.perf_counter()
    oracle.quartet_batch(B, q, tau_prim)
    dt = time.perf_counter() - t
    k = int(min(40_000_000, max(20000, 20000 * target_s / max(dt, 1e-3))))
    q = draw(k)
    t = time.perf_counter()
    oracle.quartet_batch(B, q, tau_prim)
    dt = time.perf_counter() - t
    eris = float(np.sum(nsph[q[:, 0]] * nsph[q[:, 1]] * nsph[q[:, 2]] * nsph[q[:, 3]]))
    threads = oracle.num_threads()
    # one thread on a sub-sample of about 3 s
    k1 = max(2000, int(k * min(1.0, 3.0 / max(target_s, 1e-3)) / max(threads, 1)))
    q1 = q[:k1]
    oracle.set_threads(1)
    try:
        t = time.perf_counter()
        oracle.quartet_batch(B, q1, tau_prim)
        dt1 = time.perf_counter() - t
    finally:
        oracle.set_threads(threads)
    eris1 = float(np.sum(nsph[q1[:, 0]] * nsph[q1[:, 1]] * nsph[q1[:, 2]] * nsph[q1[:, 3]]))
    return {"value": eris / dt, "unit": "ERIs/s", "cores": threads, "kind": "oracle",
            "sample": "%d uniformly drawn kept shell quartets of mol40 (each evaluated once, "
                      "spherical blocks), %.1f s" % (k, dt),
            "sample_seconds": dt, "cpu_model": _cpu_model(),
            "single_thread": {"value": eris1 / dt1, "unit": "ERIs/s", "quartets": k1, "seconds": dt1}}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _xsteps(a) -> int:
    """Timed repetitions of the side measurements (the headline keeps
    --steps): at most 3, so that the default run stays within minutes."""
    return max(1, min(a.steps, 3))


def _time(fn, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def compare_precision(jk, P, J, K, a, st):
    """The other precision on the same context: time and max |dJ|, |dK|
    against the double-precision result."""
    import torch
    other = "mixed" if a.precision == "fp64" else "fp64"
    J0, K0 = J.clone(), K.clone()
    jk.set_precision(other)
    for _ in range(max(1, a.warmup)):
        J1, K1 = jk.jk(P)
    ms = _time(lambda: jk.jk(P), _xsteps(a))
    J1, K1 = jk.jk(P)
    torch.cuda.synchronize()
    s2 = jk.stats()
    jk.set_precision(a.precision)
    dJ = float((J1 - J0).abs().max())
    dK = float((K1 - K0).abs().max())
    dE = abs(float(jk.energy(P, J1, K1)) - float(jk.energy(P, J0, K0)))
    mixed_st = s2 if other == "mixed" else st
    print("compare %s: %.1f ms dJ=%.2e dK=%.2e dE=%.2e" % (other, ms, dJ, dK, dE), file=sys.stderr, flush=True)
    return {"precision": other, "ms_per_step": ms, "value": st["eris_sph"] / (ms / 1e3),
            "max_abs_dJ_vs_fp64": dJ, "max_abs_dK_vs_fp64": dK, "abs_dE_vs_fp64": dE,
            "fp32_quartet_fraction": mixed_st["n_quartets_fp32"] / max(1, st["n_quartets"]),
            "mixed_thresh": 1e-5}


def bench_prim0(jk0, P, J, K, a, st):
    """The same workload with the primitive screen off (contracted-quartet
    Schwarz rule only): time, max |dJ|, |dK| against the default build and
    the share of primitive quartets the default screen skips."""
    import torch
    from paper_2406_14920_amd import JK, synth
    mol = synth.mol40()
    jk = JK.from_molecule(mol, prim_thresh=0.0)
    for _ in range(max(1, a.warmup)):
        jk.jk(P)
    ms = _time(lambda: jk.jk(P), _xsteps(a))
    J0, K0 = jk.jk(P)
    torch.cuda.synchronize()
    s0 = jk.stats()
    jk.close()
    dJ = float((J0 - J).abs().max())
    dK = float((K0 - K).abs().max())
    skip_k = 1.0 - st["n_prim_quartets_k"] / max(1, s0["n_prim_quartets_k"])
    skip_j = 1.0 - st["n_prim_quartets_j"] / max(1, s0["n_prim_quartets_j"])
    print("prim_thresh 0: %.1f ms dJ=%.2e dK=%.2e skipped K %.4f J %.4f" % (ms, dJ, dK, skip_k, skip_j),
          file=sys.stderr, flush=True)
    return {"prim_thresh": 0.0, "ms_per_step": ms, "max_abs_dJ_vs_default": dJ, "max_abs_dK_vs_default": dK,
            "prim_quartets_k": s0["n_prim_quartets_k"], "prim_quartets_j": s0["n_prim_quartets_j"],
            "default_skips_k": skip_k, "default_skips_j": skip_j}


def bench_tuned(jk, P, J, K, a):
    """The autotuner on the headline workload, per precision: launch shapes,
    FP32 shares and ket groupings picked from timings on this context, then
    the same build timed again (results change only in the order of
    additions, or within the mixed error)."""
    import torch
    out = {}
    for prec in ("fp64", "mixed"):
        jk.set_precision(prec)
        for _ in range(max(1, a.warmup)):
            jk.jk(P)
        ms0 = _time(lambda: jk.jk(P), _xsteps(a))
        t0 = time.perf_counter()
        tun = jk.autotune(P, reps=1)
        tune_s = time.perf_counter() - t0
        for _ in range(max(1, a.warmup)):
            jk.jk(P)
        ms1 = _time(lambda: jk.jk(P), _xsteps(a))
        J1, K1 = jk.jk(P)
        torch.cuda.synchronize()
        dK = float((K1 - K).abs().max())
        inv = sum(1 for v in abi_tuning(jk)["exchange"].values() if len(v) > 2 and v[2])
        out[prec] = {"default_ms": ms0, "tuned_ms": ms1, "autotune_s": tune_s, "max_abs_dK_vs_fp64": dK,
                     "exchange_launches_by_second_shell": inv}
        print("tuned %s: default %.1f ms -> tuned %.1f ms (autotune %.1f s, %d launches grouped by d) dK=%.1e" % (
            prec, ms0, ms1, tune_s, inv, dK), file=sys.stderr, flush=True)
    jk.set_precision(a.precision)
    return out


def abi_tuning(jk):
    from paper_2406_14920_amd import abi
    return abi.eri_get_tuning(jk.ctx)


def bench_tm62(a):
    """Transition-metal-like workload (1336 functions, exponents to 2e5):
    FP64 and mixed J+K time and the mixed error against FP64."""
    import torch
    from paper_2406_14920_amd import JK, synth
    mol = synth.tm62()
    jk = JK.from_molecule(mol)
    P = torch.tensor(mol.P, dtype=torch.float64, device="cuda")
    out = {"workload": "tm62: 2 heavy centres (3 s8, 2 p6, 3 d5, 2 f1; exponents 0.05-2e5) + 60 light atoms, "
                       "%d spherical bf, Schwarz 1e-11, primitive 1e-13" % mol.nbf}
    res = {}
    for prec in ("fp64", "mixed"):
        jk.set_precision(prec)
        for _ in range(max(1, a.warmup)):
            jk.jk(P)
        ms = _time(lambda: jk.jk(P), _xsteps(a))
        J, K = jk.jk(P)
        torch.cuda.synchronize()
        res[prec] = (ms, J, K)
        out[prec + "_ms"] = ms
    st = jk.stats()
    jk.close()
    out["eris_sph"] = st["eris_sph"]
    out["value_fp64"] = st["eris_sph"] / (res["fp64"][0] * 1e-3)
    out["mixed_speedup"] = res["fp64"][0] / res["mixed"][0]
    out["mixed_max_abs_dJ"] = float((res["mixed"][1] - res["fp64"][1]).abs().max())
    out["mixed_max_abs_dK"] = float((res["mixed"][2] - res["fp64"][2]).abs().max())
    print("tm62: fp64 %.1f ms mixed %.1f ms dJ=%.2e dK=%.2e" % (
        out["fp64_ms"], out["mixed_ms"], out["mixed_max_abs_dJ"], out["mixed_max_abs_dK"]), file=sys.stderr, flush=True)
    return out


def bench_grad(a):
    """Nuclear gradient of the 20-atom workload (jk_grad, double precision)."""
    import torch
    from paper_2406_14920_amd import JK, synth
    mol = synth.mol20()
    jk = JK.from_molecule(mol)
    P = torch.tensor(mol.P, dtype=torch.float64, device="cuda")
    g = jk.grad(P)
    ms = _time(lambda: jk.grad(P), 1)
    g = jk.grad(P).cpu().numpy()
    jk.set_precision("mixed_all")
    jk.grad(P)
    ms_m = _time(lambda: jk.grad(P), 1)
    gm = jk.grad(P).cpu().numpy()
    jk.close()
    print("grad mol20: %.1f ms |sum g|=%.1e; mixed %.1f ms max|dg|=%.1e |sum g|=%.1e" % (
        ms, np.abs(g.sum(0)).max(), ms_m, np.abs(gm - g).max(), np.abs(gm.sum(0)).max()),
        file=sys.stderr, flush=True)
    return {"workload": "mol20: 20 atoms, mol40 shell set, 420 spherical bf, Schwarz 1e-11", "ms": ms,
            "max_abs_sum_over_atoms": float(np.abs(g.sum(0)).max()), "dtype": "f64",
            "mixed": {"ms": ms_m, "max_abs_dg_vs_fp64": float(np.abs(gm - g).max()),
                      "max_abs_sum_over_atoms": float(np.abs(gm.sum(0)).max()),
                      "fp32_share": "Coulomb J-engine launches (raised bra order <= 6), tau_mix 1e-5"}}


def bench_potential(a, n_mm: int = 20000):
    """Point-charge potential V and its gradient on mol40 with its 40 nuclei
    plus n_mm QM/MM-style embedding charges (the paper's nuclear-attraction
    study uses a QM region inside many thousands of point charges)."""
    import torch
    from paper_2406_14920_amd import JK, abi, synth
    mol = synth.mol40()
    chg = np.concatenate([synth.nuclei(mol, seed=1), synth.point_charges(mol, n_mm, seed=2)])
    jk = JK.from_molecule(mol)
    c = torch.tensor(chg, dtype=torch.float64, device="cuda")
    P = torch.tensor(0.5 * (mol.P + mol.P.T), dtype=torch.float64, device="cuda")
    jk.potential(c)
    jk.potential_grad(c, P)
    steps = max(1, min(a.steps, 5))
    ms_v = _time(lambda: jk.potential(c), steps)
    ms_g = _time(lambda: jk.potential_grad(c, P), steps)
    abi.eri_set_profiling(jk.ctx, True)
    jk.potential(c)
    jk.potential_grad(c, P)
    torch.cuda.synchronize()
    prof = abi.eri_profile_read(jk.ctx)
    abi.eri_set_profiling(jk.ctx, False)
    jk.close()
    vh = [r for r in prof if r["name"].startswith("vh(")]
    pair_charge = sum(r["prim_quartets"] for r in vh)
    fl = sum(r["flops"] for r in vh)
    kms = sum(r["ms"] for r in vh)
    top = max(vh, key=lambda r: r["ms"])
    ach = top["flops"] / (top["ms"] / top["launches"] * 1e-3) / 1e12
    print("potential mol40 + %d charges: V %.2f ms (%.2f TFLOP/s over the V kernels), gradient %.2f ms" % (
        n_mm, ms_v, fl / (kms * 1e-3) / 1e12, ms_g), file=sys.stderr, flush=True)
    return {"workload": "mol40 (840 spherical bf) with its 40 nuclei + %d embedding point charges" % n_mm,
            "charges": int(chg.shape[0]), "dtype": "f64", "V_ms": ms_v, "grad_ms": ms_g,
            "pair_charge_terms": int(pair_charge), "pair_charge_terms_per_s": pair_charge / (ms_v * 1e-3),
            "V_kernels_tflops": fl / (kms * 1e-3) / 1e12,
            "V_kernels_frac_fp64_peak": fl / (kms * 1e-3) / 1e12 / PEAK_FP64_VALU,
            "top_kernel": top["name"], "top_kernel_tflops": ach}


def bench_scf(a):
    """Closed-shell SCF of mol20 with nuclei (Z in {1, 6, 7, 8}): every
    iteration a full double-precision J/K build, against the dynamic scheme
    (mixed precision with a threshold following the orbital gradient,
    incremental builds under the density-weighted screen, double precision at
    the end)."""
    import torch
    from paper_2406_14920_amd import JK, scf, synth
    mol = synth.mol20()
    nuc = synth.nuclei(mol, seed=3, even=True)
    nocc = int(round(-nuc[:, 3].sum())) // 2
    jk = JK.from_molecule(mol)
    be = scf.GPUBackend(jk, nuc)
    out = {"workload": "mol20 closed-shell SCF, %d electrons, 420 spherical bf, level shift 0.3, "
                       "overlap eigenvalues below 1e-6 dropped; converged at |dE| < 1e-8 and max orbital "
                       "gradient < 1e-5" % (2 * nocc)}
    for mode in ("fp64", "dynamic"):
        t0 = time.perf_counter()
        r = scf.rhf(be, nuc, nocc, mode=mode, max_iter=120, conv=1e-8, grad_conv=1e-5, level_shift=0.3,
                    fp64_below=1e-4)
        wall = time.perf_counter() - t0
        out[mode] = {"energy": r.energy, "converged": r.converged, "iterations": len(r.iterations),
                     "build_ms_total": r.build_ms, "wall_s": wall,
                     "mixed_iterations": sum(1 for it in r.iterations if it.precision != "fp64"),
                     "incremental_iterations": sum(1 for it in r.iterations if it.incremental),
                     "errors": [float("%.2e" % it.error) for it in r.iterations],
                     "build_ms": [round(it.build_ms, 1) for it in r.iterations]}
        print("scf %s: E %.10f converged %s, %d iterations, J/K builds %.0f ms, wall %.1f s" % (
            mode, r.energy, r.converged, len(r.iterations), r.build_ms, wall), file=sys.stderr, flush=True)
    jk.close()
    out["energy_diff"] = out["dynamic"]["energy"] - out["fp64"]["energy"]
    out["build_speedup"] = out["fp64"]["build_ms_total"] / max(out["dynamic"]["build_ms_total"], 1e-9)
    return out


def bench_grid(a):
    """Exchange-correlation grid step on mol40 with its atom-centred grid:
    density and gradient at every point, a functional's potential (Slater
    exchange for v0 and a gradient term of the same scaling for v1; the paper
    evaluates the functional outside the GPU kernels and names none), then
    the matrix sums."""
    import torch
    from paper_2406_14920_amd import JK, synth
    mol = synth.mol40()
    pts, w = synth.molecular_grid(mol)
    jk = JK.from_molecule(mol)
    P = torch.tensor(0.5 * (mol.P + mol.P.T), dtype=torch.float64, device="cuda")
    pt = torch.tensor(pts, dtype=torch.float64, device="cuda")
    wt = torch.tensor(w, dtype=torch.float64, device="cuda")

    def potential(rho, grad):
        r = torch.clamp(rho, min=1e-14)
        v0 = -(3.0 / np.pi) ** (1.0 / 3.0) * r ** (1.0 / 3.0) * wt
        v1 = (-0.0042 * grad / r[:, None] ** (4.0 / 3.0)) * wt[:, None]
        return v0.contiguous(), v1.contiguous()

    rho, grad = jk.grid_density(P, pt)
    v0, v1 = potential(rho, grad)
    jk.grid_matrix(pt, v0, v1)
    steps = max(1, min(a.steps, 5))
    ms_rho = _time(lambda: jk.grid_density(P, pt), steps)
    ms_mat = _time(lambda: jk.grid_matrix(pt, v0, v1), steps)
    n_el = float(torch.sum(wt * rho))
    jk.close()
    print("grid mol40: %d points, density+gradient %.2f ms, matrix %.2f ms, electrons %.6f (tr PS check)" % (
        pts.shape[0], ms_rho, ms_mat, n_el), file=sys.stderr, flush=True)
    return {"workload": "mol40 (840 spherical bf), atom-centred grid 40 radial x 11 x 22 angular per atom, "
                        "Becke partition", "points": int(pts.shape[0]), "dtype": "f64",
            "density_gradient_ms": ms_rho, "matrix_ms": ms_mat,
            "points_per_s_density": pts.shape[0] / (ms_rho * 1e-3), "integrated_electrons": n_el}


def _lat(b):
    lat = np.array(b.latency())
    return {"min": float(lat.min()), "median": float(np.median(lat)), "p90": float(np.percentile(lat, 90)),
            "max": float(lat.max())}


def bench_batch(a):
    """64 molecules of 5-30 atoms built as one batch: queue mode (one
    launch per kernel over every molecule's blocks) and streams
    mode (molecules on concurrent streams), against the same molecules built
    one after another; and mol40 alone as a batch of one in queue mode
    against its own build_jk."""
    import torch
    from paper_2406_14920_amd import JK, Batch, synth
    mols = synth.batch64()
    t0 = time.perf_counter()
    jks = [JK.from_molecule(m) for m in mols]
    setup_s = time.perf_counter() - t0
    Ps = [torch.tensor(m.P, dtype=torch.float64, device="cuda") for m in mols]
    eris = sum(jk.stats()["eris_sph"] for jk in jks)
    s = torch.cuda.Stream()
    b = Batch(jks, stream=s, mode="queue")
    t0 = time.perf_counter()
    b.jk(Ps)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = b.queue_info()
    ms_queue = _time(lambda: b.jk(Ps), _xsteps(a))
    lat_queue = _lat(b)
    # the same build captured once into a HIP graph and replayed
    Jq = [t.clone() for t in b.J]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.jk(Ps)
    g.replay()
    torch.cuda.synchronize()
    ms_graph = _time(g.replay, _xsteps(a))
    graph_dj = max(float((x - y).abs().max()) for x, y in zip(b.J, Jq))
    del g
    b.set_mode("streams")
    b.jk(Ps)
    ms_streams = _time(lambda: b.jk(Ps), _xsteps(a))
    lat_streams = _lat(b)
    ms_seq = _time(lambda: [jk.jk(P) for jk, P in zip(jks, Ps)], _xsteps(a))
    # FP32-mixed batch in queue mode against the FP64 results
    b.set_mode("queue")
    J64, K64 = b.jk(Ps)
    J64 = [t.clone() for t in J64]
    K64 = [t.clone() for t in K64]
    for jk in jks:
        jk.set_precision("mixed")
    b.jk(Ps)
    ms_mixed = _time(lambda: b.jk(Ps), _xsteps(a))
    lat_mixed = _lat(b)
    Jm, Km = b.jk(Ps)
    torch.cuda.synchronize()
    dj = max(float((x - y).abs().max()) for x, y in zip(Jm, J64))
    dk = max(float((x - y).abs().max()) for x, y in zip(Km, K64))
    b.close()
    for jk in jks:
        jk.close()
    print("batch64: queue %.1f ms (graph replay %.1f ms), streams %.1f ms, one by one %.1f ms, mixed (queue) %.1f ms "
          "(setup %.1fs, first queue call %.1fs)" % (ms_queue, ms_graph, ms_streams, ms_seq, ms_mixed, setup_s, plan_s),
          file=sys.stderr, flush=True)
    m40 = synth.mol40()
    jk40 = JK.from_molecule(m40)
    P40 = torch.tensor(m40.P, dtype=torch.float64, device="cuda")
    b1 = Batch([jk40], mode="queue")
    b1.jk([P40])
    ms40_queue = _time(lambda: b1.jk([P40]), _xsteps(a))
    info40 = b1.queue_info()
    ms40_direct = _time(lambda: jk40.jk(P40), _xsteps(a))
    b1.close()
    jk40.close()
    print("mol40: queue (batch of one) %.1f ms, build_jk %.1f ms" % (ms40_queue, ms40_direct),
          file=sys.stderr, flush=True)
    return {"workload": "64 molecules of 5-30 atoms (mol40 shell set), FP64", "molecules": len(mols),
            "nbf_range": [min(m.nbf for m in mols), max(m.nbf for m in mols)],
            "ms_per_batch": ms_queue, "eris_per_s_batch": eris / (ms_queue / 1e3),
            "launch": "queue mode: one launch per kernel over the blocks of all 64 molecules, "
                      "launches with the most work per block first",
            "queue_plan": {"launches": info["launches"], "items": info["items"], "first_call_s": plan_s},
            "ms_per_batch_graph_replay": ms_graph, "graph_replay_max_abs_dJ_vs_eager": graph_dj,
            "per_molecule_latency_ms": lat_queue,
            "ms_per_batch_streams": ms_streams, "per_molecule_latency_ms_streams": lat_streams,
            "ms_per_batch_one_by_one": ms_seq,
            "mixed": {"ms_per_batch": ms_mixed, "eris_per_s": eris / (ms_mixed / 1e3), "launch": "queue mode",
                      "per_molecule_latency_ms": lat_mixed, "max_abs_dJ_vs_fp64": dj, "max_abs_dK_vs_fp64": dk,
                      "mixed_thresh": 1e-5},
            "latency_of": "last timed call, from its start to each molecule's completion (HIP events)",
            "mol40_as_batch_of_one": {"queue_ms": ms40_queue, "build_jk_ms": ms40_direct,
                                      "queue_launches": info40["launches"], "queue_items": info40["items"]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--profile-json", default=None, help="write the per-kernel table here")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES bytes five times (counter calibration) and exit")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the side measurements (other precision, tm62, gradient, potential, SCF, grid, batch)")
    ap.add_argument("--only", default=None,
                    choices=["tm62", "grad", "potential", "scf", "grid", "batch"],
                    help="run only this side measurement, print its JSON and exit (for profiling one family)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if a.copy_probe:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings
        # calibrate the HBM-traffic counters of the J/K kernels
        src = torch.ones(a.copy_probe // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.copy_probe}), flush=True)
        return
    if a.only:
        fn = {"tm62": bench_tm62, "grad": bench_grad, "potential": bench_potential, "scf": bench_scf,
              "grid": bench_grid, "batch": bench_batch}[a.only]
        print(json.dumps({a.only: fn(a)}), flush=True)
        return
    from paper_2406_14920_amd import JK, abi, synth

    mol = synth.mol40()
    t0 = time.perf_counter()
    jk = JK.from_molecule(mol, precision=a.precision)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    P = torch.tensor(mol.P, dtype=torch.float64, device="cuda")
    st = jk.stats()
    print("setup %.2fs nbf=%d quartets=%d eris_sph=%.3e flopsK=%.3e flopsJ=%.3e" % (
        setup_s, st["nbf"], st["n_quartets"], st["eris_sph"], st["model_flops_k"], st["model_flops_j"]),
        file=sys.stderr, flush=True)

    for _ in range(a.warmup):
        jk.jk(P)
    torch.cuda.synchronize()

    # timed region: the concurrent path as it runs in production
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        J, K = jk.jk(P)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt / a.steps * 1e3
    value = st["eris_sph"] / (ms / 1e3)
    # profiled pass (same number of steps; the library runs it on one stream so
    # that its HIP events bracket each kernel alone): per-kernel times
    abi.eri_set_profiling(jk.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        jk.jk(P)
    torch.cuda.synchronize()
    ms_prof = (time.perf_counter() - t0) / a.steps * 1e3
    prof = abi.eri_profile_read(jk.ctx)
    abi.eri_set_profiling(jk.ctx, False)

    prof.sort(key=lambda r: -r["ms"])
    top = prof[0]
    avg_ms = top["ms"] / top["launches"]
    achieved = top["flops"] / (avg_ms * 1e-3) / 1e12
    kern_total = sum(r["ms"] for r in prof) / a.steps
    traffic = _traffic(top["name"], 1)
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VALU, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_VALU, "traffic": traffic, "kernel": top["name"],
            "kernel_avg_ms": avg_ms, "kernel_share_of_serial_step": top["ms"] / a.steps / ms_prof,
            "measured_in": "profiled pass of %d steps run on one stream after the timed region" % a.steps}
    flops_total = st["model_flops_k"] + st["model_flops_j"]
    out = {
        "metric": METRIC, "value": value, "unit": "ERIs/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if a.precision == "fp64" else "f32+f64",
        "data": "synthetic (seeded 40-atom cluster, random orthonormal density)",
        "config": {"workload": "mol40: 40 atoms, s6 s3 s1 p3 p1 d1 f1 per atom, 840 spherical bf, "
                               "Schwarz 1e-11, primitive 1e-13", "nbf": st["nbf"],
                   "quartets": st["n_quartets"], "precision": a.precision},
        "path_tflops": flops_total / (ms * 1e-3) / 1e12,
        "path_frac_fp64_peak": flops_total / (ms * 1e-3) / 1e12 / PEAK_FP64_VALU,
        "kernel_ms_per_step_serial": kern_total, "ms_per_step_serial": ms_prof,
        "roofline": roof,
    }
    if a.profile_json:
        with open(a.profile_json, "w") as f:
            json.dump({"steps": a.steps, "ms_per_step": ms, "kernels": prof}, f, indent=1)
    if not a.no_extras:
        out["compare"] = compare_precision(jk, P, J, K, a, st)
        out["prim_thresh_0"] = bench_prim0(jk, P, J, K, a, st)
        out["tuned"] = bench_tuned(jk, P, J, K, a)
    jk.close()
    if not a.no_extras:
        out["tm62"] = bench_tm62(a)
    if not a.no_extras:
        out["grad"] = bench_grad(a)
        out["potential"] = bench_potential(a)
        out["scf"] = bench_scf(a)
        out["grid"] = bench_grid(a)
        out["batch64"] = bench_batch(a)
    if not a.no_cpu:
        cb = cpu_baseline(mol)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "cpu_model",
                                                  "single_thread")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
