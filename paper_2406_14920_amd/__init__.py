"""MI355X-native direct-SCF J/K (and J/K energy gradient) library.

    from paper_2406_14920_amd import JK, synth
    mol = synth.mol40()
    jk = JK.from_molecule(mol)                  # eri_setup
    J, K = jk.jk(P)                             # build_jk, P a float64 CUDA tensor

The numerical work runs in libmdjk.so (hand-written HIP for gfx950); see
include/mdjk.h for the C ABI.  Importing this package does not load the
library; the first call that needs it does, and raises if it is missing.
"""
from __future__ import annotations

from typing import Optional, Tuple

from . import abi  # noqa: F401  (ctypes only; loads the .so lazily)

__all__ = ["abi", "JK", "JKEnergy", "Batch"]

# precision names: "fp64"; "mixed" (FP32 share where it is faster);
# "mixed_all" (the density-weighted rule on every launch)
_PREC = {"fp64": abi.ERI_FP64, "mixed": abi.ERI_MIXED, "mixed_all": abi.ERI_MIXED_ALL}


class JK:
    """One eri_ctx: a fixed basis/geometry, reused across builds."""

    def __init__(self, shells, xyz, schwarz_thresh: float = 1e-11, prim_thresh: Optional[float] = None,
                 precision: str = "fp64", mixed_thresh: float = 1e-5, spherical: bool = True,
                 stream=None, omega: float = 0.0):
        import torch
        o = abi.eri_default_opts()
        o.schwarz_thresh = float(schwarz_thresh)
        o.prim_thresh = float(1e-2 * schwarz_thresh if prim_thresh is None else prim_thresh)
        o.mixed_thresh = float(mixed_thresh)
        o.precision = _PREC[precision]
        self._precision = o.precision
        o.spherical = 1 if spherical else 0
        o.omega = float(omega)  # 0: 1/r; > 0: erf(omega r)/r
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        o.stream = int(stream.cuda_stream)
        self.opts = o
        self.natom = len(xyz)
        self._xyz = [[float(v) for v in r] for r in xyz]
        self.ctx = abi.eri_setup(shells, xyz, o)
        self.nbf = abi.eri_nbf(self.ctx)

    @classmethod
    def from_molecule(cls, mol, **kw):
        shells = [(s.atom, s.l, s.exps, s.coefs) for s in mol.shells]
        kw.setdefault("schwarz_thresh", mol.tau_schwarz)
        return cls(shells, mol.xyz, **kw)

    def jk(self, P, want_j: bool = True, want_k: bool = True) -> Tuple:
        import torch
        if P.dtype != torch.float64 or not P.is_cuda or not P.is_contiguous():
            raise ValueError("P must be a contiguous float64 CUDA tensor")
        if P.shape != (self.nbf, self.nbf):
            raise ValueError("P must be %d x %d" % (self.nbf, self.nbf))
        J = torch.empty_like(P) if want_j else None
        K = torch.empty_like(P) if want_k else None
        with torch.cuda.stream(self.stream):
            abi.build_jk(self.ctx, P, J, K)
        return J, K

    def grad(self, P, energy: bool = False):
        """dE/dR (natom x 3, hartree/bohr) of E = 1/2 tr(PJ) - 1/4 tr(PK) at
        fixed P (jk_grad); with energy=True also E (0-dim tensor)."""
        import torch
        if P.dtype != torch.float64 or not P.is_cuda or not P.is_contiguous():
            raise ValueError("P must be a contiguous float64 CUDA tensor")
        g = torch.empty((self.natom, 3), dtype=torch.float64, device=P.device)
        E = torch.empty((), dtype=torch.float64, device=P.device) if energy else None
        with torch.cuda.stream(self.stream):
            abi.jk_grad(self.ctx, P, g, E)
        return (g, E) if energy else g

    def one_electron(self):
        """(S, T): overlap and kinetic energy matrices (eri_one_electron)."""
        import torch
        S = torch.empty((self.nbf, self.nbf), dtype=torch.float64, device="cuda")
        T = torch.empty_like(S)
        with torch.cuda.stream(self.stream):
            abi.eri_one_electron(self.ctx, S, T)
        return S, T

    def _points(self, pts):
        import torch
        if pts.dtype != torch.float64 or not pts.is_cuda or not pts.is_contiguous():
            raise ValueError("points must be a contiguous float64 CUDA tensor")
        if pts.dim() != 2 or pts.shape[1] != 3:
            raise ValueError("points must be n x 3")
        return int(pts.shape[0])

    def grid_density(self, P, pts, gradient: bool = True):
        """(rho (n,), grad rho (n, 3) or None) at the points (eri_grid_density)."""
        import torch
        n = self._points(pts)
        rho = torch.empty(n, dtype=torch.float64, device=pts.device)
        grad = torch.empty((n, 3), dtype=torch.float64, device=pts.device) if gradient else None
        with torch.cuda.stream(self.stream):
            abi.eri_grid_density(self.ctx, P, pts, n, rho, grad)
        return rho, grad

    def grid_matrix(self, pts, v0, v1=None):
        """V_mn = sum_g v0_g m n + v1_g . grad(m n) (eri_grid_matrix)."""
        import torch
        n = self._points(pts)
        for name, v, shp in (("v0", v0, (n,)), ("v1", v1, (n, 3))):
            if v is not None and (v.dtype != torch.float64 or not v.is_cuda or not v.is_contiguous()
                                  or tuple(v.shape) != shp):
                raise ValueError("%s must be a contiguous float64 CUDA tensor of shape %s" % (name, shp))
        V = torch.empty((self.nbf, self.nbf), dtype=torch.float64, device=pts.device)
        with torch.cuda.stream(self.stream):
            abi.eri_grid_matrix(self.ctx, pts, n, v0, v1, V)
        return V

    def set_density_screen(self, tau: float):
        """Density-weighted screen of later builds (0: off)."""
        abi.eri_set_density_screen(self.ctx, tau)

    def _charges(self, charges):
        import torch
        if charges.dtype != torch.float64 or not charges.is_cuda or not charges.is_contiguous():
            raise ValueError("charges must be a contiguous float64 CUDA tensor")
        if charges.dim() != 2 or charges.shape[1] != 4:
            raise ValueError("charges must be n x 4 (x, y, z, q)")
        return charges, int(charges.shape[0])

    def potential(self, charges):
        """V_mn = sum_C q_C (m|1/|r - C||n) (eri_potential); charges: n x 4
        float64 CUDA tensor of x, y, z (bohr), q (nuclei: q = -Z)."""
        import torch
        c, n = self._charges(charges)
        V = torch.empty((self.nbf, self.nbf), dtype=torch.float64, device=c.device)
        with torch.cuda.stream(self.stream):
            abi.eri_potential(self.ctx, c, n, V)
        return V

    def potential_grad(self, charges, P):
        """(dE_V/dR_atoms (natom x 3), dE_V/dR_charges (n x 3)) of
        E_V = sum P_mn V_mn at fixed P (eri_potential_grad)."""
        import torch
        c, n = self._charges(charges)
        if P.dtype != torch.float64 or not P.is_cuda or not P.is_contiguous():
            raise ValueError("P must be a contiguous float64 CUDA tensor")
        if P.shape != (self.nbf, self.nbf):
            raise ValueError("P must be %d x %d" % (self.nbf, self.nbf))
        ga = torch.empty((self.natom, 3), dtype=torch.float64, device=P.device)
        gc = torch.empty((n, 3), dtype=torch.float64, device=P.device)
        with torch.cuda.stream(self.stream):
            abi.eri_potential_grad(self.ctx, c, n, P, ga, gc if n > 0 else None)
        return ga, gc

    def energy(self, P, J, K):
        """E = 1/2 <P,J> - 1/4 <P,K> on the device (eri_energy)."""
        import torch
        E = torch.empty((), dtype=torch.float64, device=P.device)
        with torch.cuda.stream(self.stream):
            abi.eri_energy(self.ctx, P, J, K, E)
        return E

    def autotune(self, P, reps: int = 2, cache: Optional[str] = None, key: Optional[str] = None) -> dict:
        """Pick launch shapes for this workload (eri_autotune); returns them.
        With `cache` (a JSON file path), a choice saved there under `key`
        and this precision is applied instead of timing, and a new choice is
        saved there."""
        import json
        import os
        ck = "%s/%s" % (key or "nbf%d" % self.nbf, self.precision_name())
        store = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                store = json.load(f)
            if ck in store:
                abi.eri_set_tuning(self.ctx, store[ck])
                return abi.eri_tuning(self.ctx)
        with __import__("torch").cuda.stream(self.stream):
            abi.eri_autotune(self.ctx, P, reps)
        if cache:
            store[ck] = abi.eri_get_tuning(self.ctx)
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(store, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return abi.eri_tuning(self.ctx)

    def precision_name(self) -> str:
        return {v: k for k, v in _PREC.items()}[self._precision]

    def set_geometry(self, xyz):
        """Move the atoms (same shells); redoes pair setup (synchronous)."""
        abi.eri_set_geometry(self.ctx, xyz)
        self._xyz = [[float(v) for v in r] for r in xyz]

    def set_precision(self, precision: str, mixed_thresh: Optional[float] = None):
        abi.eri_set_precision(self.ctx, _PREC[precision],
                              self.opts.mixed_thresh if mixed_thresh is None else mixed_thresh)
        self._precision = _PREC[precision]

    def set_omega(self, omega: float):
        """Two-electron operator of later builds: 0 for 1/r, > 0 for erf(omega r)/r."""
        abi.eri_set_omega(self.ctx, omega)

    def stats(self) -> dict:
        return abi.eri_stats(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            abi.eri_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many JK contexts built together (eri_batch_*).  mode "queue" (the
    default): one launch per kernel (and arithmetic type) for the whole
    batch, whose workgroups run the blocks of every molecule's launch from a
    device-side work list, most work first; mode "streams": every molecule's build forked from the batch
    stream onto one of a few streams, largest first, and joined back.
    Output tensors are allocated once and reused."""

    MODES = {"queue": abi.ERI_BATCH_QUEUE, "streams": abi.ERI_BATCH_STREAMS}

    def __init__(self, jks, stream=None, mode: str = "queue"):
        import torch
        self.jks = list(jks)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.handle = abi.eri_batch_create([j.ctx for j in self.jks], int(stream.cuda_stream))
        self.set_mode(mode)
        self.J = [torch.empty((j.nbf, j.nbf), dtype=torch.float64, device="cuda") for j in self.jks]
        self.K = [torch.empty((j.nbf, j.nbf), dtype=torch.float64, device="cuda") for j in self.jks]

    def jk(self, Ps):
        """Ps: one contiguous float64 CUDA tensor per molecule.  Returns the
        lists (J, K); their tensors are overwritten by the next call."""
        import torch
        for j, P in zip(self.jks, Ps):
            if P.dtype != torch.float64 or not P.is_cuda or not P.is_contiguous() or P.shape != (j.nbf, j.nbf):
                raise ValueError("each P must be a contiguous float64 CUDA tensor of its molecule's size")
        with torch.cuda.stream(self.stream):
            abi.eri_batch_build_jk(self.handle, list(Ps), self.J, self.K)
        return self.J, self.K

    def latency(self):
        """Per-molecule completion times (ms) of the last jk() call, from
        its start on the batch stream (eri_batch_latency)."""
        return abi.eri_batch_latency(self.handle, len(self.jks))

    def set_mode(self, mode: str):
        if mode not in self.MODES:
            raise ValueError("mode must be one of %s" % sorted(self.MODES))
        abi.eri_batch_set_mode(self.handle, self.MODES[mode])
        self.mode = mode

    def queue_info(self) -> dict:
        """Launches per build and work items of the current queue plan."""
        return abi.eri_batch_queue_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            abi.eri_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _jk_energy_class():
    import torch

    class JKEnergy(torch.autograd.Function):
        """E(coords, P) = 1/2 tr(PJ) - 1/4 tr(PK) with J, K from build_jk.

        coords: (natom, 3) float64 tensor (bohr); P: (nbf, nbf) float64 CUDA
        tensor; jk: a JK context for the same shells.  backward returns
        dE/dcoords from jk_grad (P held fixed, SI eq. si_dE_J / si_dE_K) and
        dE/dP = J - K/2.
        """

        @staticmethod
        def forward(ctx, coords, P, jk):
            xyz = coords.detach().to("cpu", torch.float64).tolist()
            if xyz != jk._xyz:
                jk.set_geometry(xyz)
            J, K = jk.jk(P)
            E = jk.energy(P, J, K)
            ctx.jk = jk
            ctx.xyz = xyz  # the context may have moved by the time backward runs
            ctx.coords_device = coords.device
            ctx.save_for_backward(P, J, K)
            return E

        @staticmethod
        def backward(ctx, gE):
            P, J, K = ctx.saved_tensors
            gc = gP = None
            if ctx.needs_input_grad[0]:
                if ctx.jk._xyz != ctx.xyz:
                    ctx.jk.set_geometry(ctx.xyz)
                gc = (ctx.jk.grad(P) * gE).to(ctx.coords_device)
            if ctx.needs_input_grad[1]:
                gP = (J - 0.5 * K) * gE
            return gc, gP, None

    return JKEnergy


class _LazyJKEnergy:
    """torch.autograd.Function built on first use (importing this package
    does not import torch)."""
    _cls = None

    def __getattr__(self, name):
        if _LazyJKEnergy._cls is None:
            _LazyJKEnergy._cls = _jk_energy_class()
        return getattr(_LazyJKEnergy._cls, name)


JKEnergy = _LazyJKEnergy()
