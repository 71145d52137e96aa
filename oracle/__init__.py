"""CPU oracle for the direct-SCF J/K build and its nuclear gradient.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The GPU library never imports it and it never
imports the GPU library.  See oracle.c for the equations it follows.

Parity status per function (what pins it is listed in tests/test_oracle_*.py):
  boys          pinned (mpmath 1F1 values, closed forms)
  e_coeffs      pinned (1D overlap by exact Gauss-Hermite quadrature)
  r_tensor      pinned (numerical derivatives of (-2a)^m F_m(a|L|^2))
  prim_block    pinned ((ss|ss) closed form, brute-force Gaussian-transform
                quadrature for l <= 3 on four centres, 8-fold symmetry)
  prim_bounds   pinned (s-s primitive pairs against the mpmath closed form of
                (ss|ss); equal to the contracted Schwarz factor for
                one-primitive shells of every l <= 3; the J/K change from
                skipping primitive quartets stays inside their Schwarz bounds)
  jk / blocks   pinned (symmetry, Coulomb-metric positivity, translation and
                rotation invariance, large-separation limit)
  grad          pinned (central finite differences of the oracle energy,
                zero sum over atoms, analytic two-centre derivative)
  vmatrix       pinned ((s|1/r_C|s) closed form of eq. v1e_base_case with
                mpmath erf; blocks up to (f|f) against a Gaussian-transform
                quadrature; far-field limit q S/|P-C|)
  vgrad         pinned (central differences of E_V in atom and charge
                positions; atom and charge derivatives sum to zero)
  ao_values,    pinned (sum_g w_g m n over a product Gauss-Legendre box grid
  grid_density, against the overlap S; gradients against central
  xc_matrix     differences; sum_g w_g grad(m n) over the box grid vanishes)
  spherical     convention pinned by S_sph = I and rotation invariance
  omega > 0     pinned (erf(omega r)/r blocks against the Gaussian-transform
                quadrature cut at t = omega and an mpmath closed form of the
                attenuated (ss|ss); the large-omega limit is the 1/r result)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence, Tuple

import numpy as np

from . import basis as _basis

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_oracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.oracle_boys.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.oracle_e_coeffs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, dp]
        L.oracle_r_tensor.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L.oracle_prim_block.argtypes = [ctypes.c_int] * 4 + [dp, dp, dp]
        bas = [ctypes.c_int32, ctypes.c_int32, ip, ip, ip, ip, dp, dp, dp]
        L.oracle_shell_block.argtypes = bas + [ctypes.c_int] * 6 + [dp]
        L.oracle_schwarz.argtypes = bas + [dp]
        qp = [dp, ctypes.c_int32, ctypes.c_double]
        L.oracle_prim_bounds.argtypes = bas + [dp]
        L.oracle_jk.argtypes = bas + [dp, ip, ip, ctypes.c_int32, dp, dp] + qp + [ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_jk_blocks.argtypes = bas + [dp, ip, ip, ctypes.c_int32, dp, dp] + qp + [ctypes.c_double,
                                             ctypes.c_int, ip, ctypes.c_int, ip,
                                             ctypes.POINTER(ctypes.c_int64), dp]
        L.oracle_grad.argtypes = bas + [dp, ip, ip, ctypes.c_int32, dp, dp] + qp + [ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        L.oracle_quartet_batch.argtypes = bas + [dp, ip] + qp + [ctypes.c_int64, ip]
        L.oracle_quartet_batch.restype = ctypes.c_double
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_vmatrix.argtypes = bas + [dp, ip, ip, ctypes.c_int32, ctypes.c_int32, dp, dp]
        L.oracle_vgrad.argtypes = bas + [dp, ip, ip, ctypes.c_int32, ctypes.c_int32, dp, dp, dp, dp]
        L.oracle_prim_vblock.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int32, dp, dp]
        L.oracle_st.argtypes = bas + [dp, ip, ip, ctypes.c_int32, dp, dp]
        L.oracle_prim_stblock.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp]
        L.oracle_set_omega.argtypes = [ctypes.c_double]
        L.oracle_set_omega.restype = None
        L.oracle_get_omega.restype = ctypes.c_double
        _lib = L
    return _lib


class _Omega:
    """Context: the two-electron operator erf(omega r)/r (omega > 0) or 1/r
    (omega = 0) for the oracle calls inside it (eqs. eri_longrange_definition,
    eri_longrange_formula)."""

    def __init__(self, omega: float):
        self.omega = float(omega)

    def __enter__(self):
        self.saved = lib().oracle_get_omega()
        lib().oracle_set_omega(self.omega)

    def __exit__(self, *exc):
        lib().oracle_set_omega(self.saved)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


# ---------------------------------------------------------------------------
# primitives exposed for the pins
# ---------------------------------------------------------------------------
def boys(mmax: int, T: float) -> np.ndarray:
    F = np.zeros(mmax + 1)
    lib().oracle_boys(mmax, float(T), _dp(F))
    return F


def e_coeffs(la, lb, a, b, Ax, Bx) -> np.ndarray:
    out = np.zeros((la + 1) * (lb + 1) * (la + lb + 1))
    lib().oracle_e_coeffs(la, lb, a, b, Ax, Bx, _dp(out))
    return out.reshape(la + 1, lb + 1, la + lb + 1)


def r_tensor(Lt: int, alpha: float, L) -> np.ndarray:
    n = Lt + 1
    out = np.zeros(n ** 3)
    Lv = np.ascontiguousarray(L, dtype=float)
    lib().oracle_r_tensor(Lt, alpha, _dp(Lv), _dp(out))
    return out.reshape(n, n, n)


def prim_block(ls, exps, centres, omega: float = 0.0) -> np.ndarray:
    """Primitive Cartesian ERI block of unnormalised monomials (operator
    erf(omega r)/r if omega > 0, else 1/r)."""
    la, lb, lc, ld = ls
    nc = [(l + 1) * (l + 2) // 2 for l in ls]
    out = np.zeros(int(np.prod(nc)))
    e = np.ascontiguousarray(exps, float)
    c = np.ascontiguousarray(centres, float).reshape(12)
    with _Omega(omega):
        lib().oracle_prim_block(la, lb, lc, ld, _dp(e), _dp(c), _dp(out))
    return out.reshape(nc)


# ---------------------------------------------------------------------------
# basis marshalling
# ---------------------------------------------------------------------------
class OBasis:
    """Flat arrays of one molecule for the C oracle."""

    def __init__(self, mol):
        self.mol = mol
        sh = mol.shells
        self.nshell = len(sh)
        self.natom = mol.natom
        self.atom = np.array([s.atom for s in sh], np.int32)
        self.l = np.array([s.l for s in sh], np.int32)
        self.nprim = np.array([len(s.exps) for s in sh], np.int32)
        self.off = np.concatenate([[0], np.cumsum(self.nprim)[:-1]]).astype(np.int32)
        self.exps = np.concatenate([np.asarray(s.exps, float) for s in sh])
        self.coefs = np.concatenate([_basis.normalised_coefs(s.l, s.exps, s.coefs) for s in sh])
        self.xyz = np.ascontiguousarray(mol.xyz, float).reshape(-1)
        self.ao_off = np.concatenate([[0], np.cumsum(2 * self.l + 1)[:-1]]).astype(np.int32)
        self.nbf = int(np.sum(2 * self.l + 1))
        Ts, offs, o = [], [], 0
        for lv in range(5):
            T = _basis.SPH[lv]
            Ts.append(T.reshape(-1))
            offs.append(o)
            o += T.size
        self.T = np.concatenate(Ts)
        self.Toff = np.array(offs, np.int32)
        self._Q = None
        self._qp = None

    def args(self):
        return (self.nshell, self.natom, _ip(self.atom), _ip(self.l), _ip(self.nprim),
                _ip(self.off), _dp(self.exps), _dp(self.coefs), _dp(self.xyz))

    def shell_block(self, a, b, c, d, dcen=-1, dax=0) -> np.ndarray:
        ls = [int(self.l[x]) for x in (a, b, c, d)]
        nc = [(l + 1) * (l + 2) // 2 for l in ls]
        out = np.zeros(int(np.prod(nc)))
        lib().oracle_shell_block(*self.args(), a, b, c, d, dcen, dax, _dp(out))
        return out.reshape(nc)

    def shell_block_sph(self, a, b, c, d) -> np.ndarray:
        blk = self.shell_block(a, b, c, d)
        for k, x in enumerate((a, b, c, d)):
            T = _basis.SPH[int(self.l[x])]
            blk = np.moveaxis(np.tensordot(T, blk, axes=([1], [k])), 0, k)
        return blk

    def prim_bounds(self) -> np.ndarray:
        """q_ij = |C_i C_j| sqrt(max |(ij|ij)|) for every pair of primitives."""
        if self._qp is None:
            n = int(self.exps.size)
            q = np.zeros((n, n))
            with _Omega(0.0):  # screening bounds of 1/r, whatever the operator
                lib().oracle_prim_bounds(*self.args(), _dp(q))
            self._qp = q
        return self._qp

    def screen_args(self, tau_prim: float):
        q = self.prim_bounds()
        return (_dp(q), int(q.shape[0]), float(tau_prim))

    def schwarz(self) -> np.ndarray:
        if self._Q is None:
            Q = np.zeros((self.nshell, self.nshell))
            with _Omega(0.0):
                lib().oracle_schwarz(*self.args(), _dp(Q))
            self._Q = Q
        return self._Q


def _sym(P):
    P = np.ascontiguousarray(P, float)
    return np.ascontiguousarray(0.5 * (P + P.T))


def _tau_prim(tau, tau_prim):
    return 1e-2 * tau if tau_prim is None else tau_prim


def jk(mol, P=None, tau=None, want_j=True, want_k=True, tau_prim=None,
       basis_obj=None, omega: float = 0.0) -> Tuple[np.ndarray, np.ndarray]:
    """Full J and K (spherical basis) by the plain definition; operator
    erf(omega r)/r if omega > 0 (screening by the 1/r bounds)."""
    B = basis_obj or OBasis(mol)
    P = _sym(mol.P if P is None else P)
    tau = mol.tau_schwarz if tau is None else tau
    Q = B.schwarz()
    J = np.zeros((B.nbf, B.nbf))
    K = np.zeros((B.nbf, B.nbf))
    sa = B.screen_args(_tau_prim(tau, tau_prim))
    with _Omega(omega):
        lib().oracle_jk(*B.args(), _dp(B.T), _ip(B.Toff), _ip(B.ao_off), B.nbf, _dp(P), _dp(Q),
                        *sa, float(tau), int(want_j), int(want_k), _dp(J), _dp(K))
    return J, K


def jk_blocks(mol, jpairs: Sequence[Tuple[int, int]], kpairs: Sequence[Tuple[int, int]],
              P=None, tau=None, basis_obj=None, tau_prim=None, omega: float = 0.0):
    """Shell blocks J[a,b] and K[a,c] for sampled shell pairs."""
    B = basis_obj or OBasis(mol)
    P = _sym(mol.P if P is None else P)
    tau = mol.tau_schwarz if tau is None else tau
    Q = B.schwarz()
    jp = np.ascontiguousarray(np.asarray(jpairs, np.int32).reshape(-1, 2))
    kp = np.ascontiguousarray(np.asarray(kpairs, np.int32).reshape(-1, 2))
    sizes = [(2 * B.l[x] + 1) * (2 * B.l[y] + 1) for x, y in list(jp) + list(kp)]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if sizes else np.zeros(0, np.int64)
    out = np.zeros(int(sum(sizes)) if sizes else 1)
    sa = B.screen_args(_tau_prim(tau, tau_prim))
    with _Omega(omega):
        lib().oracle_jk_blocks(*B.args(), _dp(B.T), _ip(B.Toff), _ip(B.ao_off), B.nbf, _dp(P), _dp(Q),
                               *sa, float(tau), len(jp), _ip(jp), len(kp), _ip(kp),
                               offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(out))
    res = []
    for t, (x, y) in enumerate(list(jp) + list(kp)):
        nx, ny = 2 * B.l[x] + 1, 2 * B.l[y] + 1
        res.append(out[offs[t]:offs[t] + nx * ny].reshape(nx, ny))
    return res[:len(jp)], res[len(jp):]


def _charges(charges):
    c = np.ascontiguousarray(np.asarray(charges, float).reshape(-1, 4))
    return c, int(c.shape[0])


def prim_vblock(ls, exps, centres, charges) -> np.ndarray:
    """Primitive Cartesian block of sum_C q_C/|r - C| between unnormalised
    monomial Gaussians (charges: rows x, y, z, q)."""
    la, lb = ls
    c, n = _charges(charges)
    out = np.zeros(((la + 1) * (la + 2) // 2) * ((lb + 1) * (lb + 2) // 2))
    e = np.ascontiguousarray(exps, float)
    x = np.ascontiguousarray(centres, float).reshape(6)
    lib().oracle_prim_vblock(la, lb, _dp(e), _dp(x), n, _dp(c), _dp(out))
    return out.reshape((la + 1) * (la + 2) // 2, (lb + 1) * (lb + 2) // 2)


def vmatrix(mol, charges, basis_obj=None) -> np.ndarray:
    """V_mn = sum_C q_C int m n / |r - C| (spherical basis), eqs. v1e_definition,
    v1e_formula; charges: rows x, y, z, q (nuclei: q = -Z)."""
    B = basis_obj or OBasis(mol)
    c, n = _charges(charges)
    V = np.zeros((B.nbf, B.nbf))
    lib().oracle_vmatrix(*B.args(), _dp(B.T), _ip(B.Toff), _ip(B.ao_off), B.nbf, n, _dp(c), _dp(V))
    return V


def vgrad(mol, charges, P=None, basis_obj=None):
    """dE_V/dR of E_V = sum P_mn V_mn at fixed P: (per atom carrying basis
    functions, per charge position), SI eqs. si_v1e_derivative_A/B/C."""
    B = basis_obj or OBasis(mol)
    c, n = _charges(charges)
    P = _sym(mol.P if P is None else P)
    ga = np.zeros((B.natom, 3))
    gc = np.zeros((max(n, 1), 3))
    lib().oracle_vgrad(*B.args(), _dp(B.T), _ip(B.Toff), _ip(B.ao_off), B.nbf, n, _dp(c), _dp(P), _dp(ga), _dp(gc))
    return ga, gc[:n]


def prim_stblock(ls, exps, centres):
    """Primitive Cartesian overlap and kinetic blocks between unnormalised
    monomial Gaussians (eqs. overlap_formula, kinetic_formula)."""
    la, lb = ls
    n = ((la + 1) * (la + 2) // 2, (lb + 1) * (lb + 2) // 2)
    S = np.zeros(n[0] * n[1])
    T = np.zeros(n[0] * n[1])
    e = np.ascontiguousarray(exps, float)
    x = np.ascontiguousarray(centres, float).reshape(6)
    lib().oracle_prim_stblock(la, lb, _dp(e), _dp(x), _dp(S), _dp(T))
    return S.reshape(n), T.reshape(n)


def st(mol, basis_obj=None):
    """Overlap S and kinetic energy T (spherical basis) over every ordered
    shell pair (eqs. overlap_definition, kinetic_definition)."""
    B = basis_obj or OBasis(mol)
    S = np.zeros((B.nbf, B.nbf))
    T = np.zeros((B.nbf, B.nbf))
    lib().oracle_st(*B.args(), _dp(B.T), _ip(B.Toff), _ip(B.ao_off), B.nbf, _dp(S), _dp(T))
    return S, T


def nuclear_repulsion(charges) -> float:
    """sum over pairs of point charges q_A q_B / |A - B|."""
    c = np.asarray(charges, float).reshape(-1, 4)
    e = 0.0
    for i in range(c.shape[0]):
        for j in range(i):
            e += c[i, 3] * c[j, 3] / np.linalg.norm(c[i, :3] - c[j, :3])
    return e


def rhf(mol, nuclei, nocc: int, conv: float = 1e-10, max_iter: int = 200, basis_obj=None, tau=None,
        tau_prim=None):
    """Closed-shell Hartree-Fock energy: F = T + V + J(P) - K(P)/2 with the
    total density P = 2 C_occ C_occ^T (J, K by eqs. j_definition and
    k_definition; V of the nuclei q = -Z by eq. v1e_definition), solved in the
    canonically orthogonalised basis (overlap eigenvalues below 1e-8 dropped)
    with Pulay's commutator extrapolation, from the core-Hamiltonian guess.
    Returns (E_total, P, iterations)."""
    B = basis_obj or OBasis(mol)
    S, T = st(mol, basis_obj=B)
    H = T + vmatrix(mol, nuclei, basis_obj=B)
    s, U = np.linalg.eigh(S)
    keep = s > 1e-8
    X = U[:, keep] / np.sqrt(s[keep])
    enuc = nuclear_repulsion(nuclei)

    def density(F):
        e, C = np.linalg.eigh(X.T @ F @ X)
        Co = X @ C[:, :nocc]
        return 2.0 * Co @ Co.T

    P = density(H)
    Fs, errs = [], []
    E_old = None
    for it in range(1, max_iter + 1):
        J, K = jk(mol, P=P, basis_obj=B, tau=tau, tau_prim=tau_prim)
        F = H + J - 0.5 * K
        E = 0.5 * float(np.sum(P * (H + F))) + enuc
        err = X.T @ (F @ P @ S - S @ P @ F) @ X
        Fs.append(F)
        errs.append(err)
        Fs, errs = Fs[-8:], errs[-8:]
        if E_old is not None and abs(E - E_old) < conv and np.abs(err).max() < 1e-7:
            return E, P, it
        E_old = E
        n = len(Fs)
        Bm = -np.ones((n + 1, n + 1))
        Bm[n, n] = 0.0
        for i in range(n):
            for j in range(n):
                Bm[i, j] = float(np.sum(errs[i] * errs[j]))
        rhs = np.zeros(n + 1)
        rhs[n] = -1.0
        c = np.linalg.lstsq(Bm, rhs, rcond=None)[0][:n]
        P = density(sum(ci * Fi for ci, Fi in zip(c, Fs)))
    raise RuntimeError("rhf: no convergence in %d iterations" % max_iter)


def ao_values(mol, pts, deriv: bool = False, basis_obj=None):
    """Basis functions at points (spherical basis, nbf x npts) and, with
    deriv, their gradients (3 x nbf x npts): every contracted Cartesian
    Gaussian sum_k c_k x_A^i y_A^j z_A^l e^{-a_k |r - A|^2} (eqs.
    contracted_basis, primtive_basis) written out at each point, then the
    spherical transform; d/dx x_A^i e^{-a r_A^2} = i x_A^{i-1} e - 2a x_A^{i+1} e."""
    B = basis_obj or OBasis(mol)
    pts = np.asarray(pts, float).reshape(-1, 3)
    n = pts.shape[0]
    chi = np.zeros((B.nbf, n))
    dchi = np.zeros((3, B.nbf, n)) if deriv else None
    for s in range(B.nshell):
        l, at, o, npr = int(B.l[s]), int(B.atom[s]), int(B.off[s]), int(B.nprim[s])
        d = pts - B.xyz[3 * at:3 * at + 3]
        r2 = np.sum(d * d, axis=1)
        g = np.zeros(n)
        gp = np.zeros(n)  # d g / d(r^2) times 2: the radial factor of the derivative
        for k in range(npr):
            ek = np.exp(-B.exps[o + k] * r2) * B.coefs[o + k]
            g += ek
            gp += -2.0 * B.exps[o + k] * ek
        comps = _basis.cart_list(l)
        cart = np.array([d[:, 0] ** i * d[:, 1] ** j * d[:, 2] ** m * g for (i, j, m) in comps])
        T = _basis.SPH[l]
        a0 = int(B.ao_off[s])
        chi[a0:a0 + 2 * l + 1] = T @ cart
        if deriv:
            for ax in range(3):
                rows = []
                for c in comps:
                    pw = list(c)
                    mono = np.prod([d[:, q] ** pw[q] for q in range(3)], axis=0)
                    lower = 0.0
                    if pw[ax] > 0:
                        pm = list(pw)
                        pm[ax] -= 1
                        lower = pw[ax] * np.prod([d[:, q] ** pm[q] for q in range(3)], axis=0) * g
                    rows.append(lower + mono * d[:, ax] * gp)
                dchi[ax, a0:a0 + 2 * l + 1] = T @ np.array(rows)
    return (chi, dchi) if deriv else chi


def grid_density(mol, P, pts, basis_obj=None):
    """rho(r_g) = sum P_mn m(r_g) n(r_g) and its gradient (eqs. xc_density_0,
    xc_density_1) at every point: (npts,), (npts, 3)."""
    chi, dchi = ao_values(mol, pts, deriv=True, basis_obj=basis_obj)
    Ps = _sym(P)
    Pc = Ps @ chi
    rho = np.sum(chi * Pc, axis=0)
    grad = 2.0 * np.einsum("kmg,mg->gk", dchi, Pc)
    return rho, grad


def xc_matrix(mol, pts, v0, v1=None, basis_obj=None):
    """V_mn = sum_g v0_g m(r_g) n(r_g) + sum_g v1_g . grad(m n)(r_g)
    (eqs. xc_grid_sum_0, xc_grid_sum_1, the weights folded into v0, v1)."""
    chi, dchi = ao_values(mol, pts, deriv=True, basis_obj=basis_obj)
    V = (chi * np.asarray(v0, float)[None, :]) @ chi.T
    if v1 is not None:
        v1 = np.asarray(v1, float).reshape(-1, 3)
        for k in range(3):
            W = (dchi[k] * v1[None, :, k]) @ chi.T
            V += W + W.T
    return V


def energy(mol, J, K, P=None) -> float:
    """E = 1/2 tr(PJ) - 1/4 tr(PK)  (SI eq. si_E_J_K)."""
    P = _sym(mol.P if P is None else P)
    return 0.5 * float(np.sum(P * J)) - 0.25 * float(np.sum(P * K))


def grad(mol, P=None, tau=None, wj=1.0, wk=1.0, only_atom=-1, Q=None, tau_prim=None,
         qprim=None, omega: float = 0.0) -> np.ndarray:
    """dE/dR (natom x 3) of E = wj/2 tr(PJ) - wk/4 tr(PK) at fixed P."""
    B = OBasis(mol)
    if qprim is not None:
        B._qp = np.ascontiguousarray(qprim, float)
    P = _sym(mol.P if P is None else P)
    tau = mol.tau_schwarz if tau is None else tau
    Q = B.schwarz() if Q is None else np.ascontiguousarray(Q, float)
    g = np.zeros((B.natom, 3))
    sa = B.screen_args(_tau_prim(tau, tau_prim))
    with _Omega(omega):
        lib().oracle_grad(*B.args(), _dp(B.T), _ip(B.Toff), _ip(B.ao_off), B.nbf, _dp(P), _dp(Q),
                          *sa, float(tau), float(wj), float(wk), int(only_atom), _dp(g))
    return g


def quartet_batch(B: "OBasis", quartets, tau_prim: float) -> float:
    """Evaluate the spherical blocks of shell quartets [(a,b,c,d), ...] (checksum)."""
    q4 = np.ascontiguousarray(np.asarray(quartets, np.int32).reshape(-1, 4))
    return float(lib().oracle_quartet_batch(*B.args(), _dp(B.T), _ip(B.Toff), *B.screen_args(tau_prim),
                                            int(q4.shape[0]), _ip(q4)))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (timing only)."""
    lib().oracle_set_threads(int(n))


sph_matrix = _basis.sph_matrix
normalised_coefs = _basis.normalised_coefs
cart_list = _basis.cart_list
