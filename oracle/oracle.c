/*
 * oracle.c -- plain, slow FP64 CPU reference for McMurchie-Davidson electron
 * repulsion integrals, direct Coulomb/exchange matrices and the nuclear
 * gradient of E = 1/2 tr(PJ) - 1/4 tr(PK).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library includes, links or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code with the GPU path.
 *
 * Every step follows the paper's theory section in its own order and notation
 * (arXiv 2406.14920, section "Theory"):
 *   - Boys function F_m(x) = int_0^1 t^{2m} exp(-x t^2) dt       (eq. boys_function)
 *   - Hermite expansion coefficients E^{ij}_t by the MD recurrence (eq. E_recursion;
 *     the right-hand factor of eq. cartesian_to_hermite is read as (tau-B)^{j})
 *   - auxiliary integrals R^m_{tuv} by their recurrence           (eq. R_recursion)
 *   - ERI as sum_P E_P sum_Q E_Q (-1)^{|Q|} 2 pi^{5/2}/(pq sqrt(p+q)) R_{P+Q}
 *     (eq. eri_formula; the ket E uses the ket exponent q)
 *   - J_{mn} = sum_{ls} (mn|ls) D_{ls}, K_{ml} = sum_{ns} (mn|ls) D_{ns}
 *     (eqs. j_definition, k_definition), written out over ordered shell quartets
 *   - E_J, E_K and their nuclear derivatives (SI eqs. si_E_J_K, si_dE_J_step1,
 *     si_dE_K_step1) by differentiating every basis function centre:
 *     d/dA_x [(x-A_x)^i e^{-a(x-A_x)^2}] = 2a (x-A_x)^{i+1} e - i (x-A_x)^{i-1} e.
 *
 * The range-separated operator erf(omega r)/r (eqs. eri_longrange_definition,
 * eri_longrange_formula) replaces 1/r when oracle_set_omega(omega > 0) is in
 * effect; the screening bounds are always those of 1/r (see oracle/__init__.py).
 *
 * The screening rule is part of the result's definition: a shell quartet
 * (ab|cd) enters iff Q_ab * Q_cd >= tau, with Q_ab = sqrt(max over Cartesian
 * components of |(ab|ab)|) (eq. cauchy_schwarz_bound at contracted-shell level);
 * inside a kept shell quartet a primitive quartet enters iff q_ij * q_kl >= tau_prim,
 * q_ij being the same bound for one primitive pair with its coefficients (the
 * paper screens pGTO pairs by this bound, section "Data structure").  Q_ab itself
 * is taken over every primitive.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC oracle.c -o _oracle.so -lm
 * (no -ffast-math, no FMA contraction flags).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXL 5                 /* shell l up to 4 (+1 inside derivatives) */
#define OR_MAXLT (4 * OR_MAXL + 1) /* max total Hermite order + 1 */
#define OR_PI 3.14159265358979323846264338327950288

/* ------------------------------------------------------------------------ */
/* Boys function                                                            */
/* ------------------------------------------------------------------------ */

/* F_m(T) for m = 0..mmax.  For T <= 50: the convergent all-positive series
 *   F_m(T) = e^{-T} sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)),
 * evaluated independently for every m.  For T > 50: F_0 = 1/2 sqrt(pi/T) erf(sqrt T)
 * and the upward recursion F_{m+1} = ((2m+1) F_m - e^{-T}) / (2T), which is
 * stable because m < T there. */
void oracle_boys(int mmax, double T, double *F)
{
    if (T <= 50.0) {
        double eT = exp(-T);
        for (int m = 0; m <= mmax; ++m) {
            double term = 1.0 / (2 * m + 1), sum = term;
            for (int k = 1; k < 2000; ++k) {
                term *= 2.0 * T / (2 * m + 2 * k + 1);
                sum += term;
                if (term < 1e-18 * sum) break;
            }
            F[m] = eT * sum;
        }
    } else {
        double eT = exp(-T);
        F[0] = 0.5 * sqrt(OR_PI / T) * erf(sqrt(T));
        for (int m = 0; m < mmax; ++m)
            F[m + 1] = ((2 * m + 1) * F[m] - eT) / (2.0 * T);
    }
}

/* ------------------------------------------------------------------------ */
/* Hermite expansion coefficients, one Cartesian direction (eq. E_recursion) */
/* E[i][j][t], i <= la, j <= lb, 0 <= t <= i+j                               */
/* ------------------------------------------------------------------------ */
typedef double etab_t[OR_MAXL + 2][OR_MAXL + 2][2 * OR_MAXL + 4];

static void e_coeffs(int la, int lb, double a, double b, double Ax, double Bx, etab_t E)
{
    double p = a + b;
    double Px = (a * Ax + b * Bx) / p;
    double XPA = Px - Ax, XPB = Px - Bx;
    double o2p = 1.0 / (2.0 * p);
    memset(E, 0, sizeof(etab_t));
    E[0][0][0] = exp(-a * b / p * (Ax - Bx) * (Ax - Bx));
    /* raise i with j = 0 */
    for (int i = 0; i < la; ++i)
        for (int t = 0; t <= i + 1; ++t) {
            double v = XPA * E[i][0][t];
            if (t > 0) v += o2p * E[i][0][t - 1];
            if (t + 1 <= i) v += (t + 1) * E[i][0][t + 1];
            E[i + 1][0][t] = v;
        }
    /* raise j for every i */
    for (int i = 0; i <= la; ++i)
        for (int j = 0; j < lb; ++j)
            for (int t = 0; t <= i + j + 1; ++t) {
                double v = XPB * E[i][j][t];
                if (t > 0) v += o2p * E[i][j][t - 1];
                if (t + 1 <= i + j) v += (t + 1) * E[i][j][t + 1];
                E[i][j + 1][t] = v;
            }
}

/* ------------------------------------------------------------------------ */
/* Auxiliary integrals R^0_{tuv}(alpha, L) for t+u+v <= Lt (eq. R_recursion) */
/* ------------------------------------------------------------------------ */
typedef struct { double v[OR_MAXLT][OR_MAXLT][OR_MAXLT]; } rtab_t;

static void r_tensor(int Lt, double alpha, const double L[3], rtab_t *R0, rtab_t *work)
{
    double F[OR_MAXLT + 1];
    double T = alpha * (L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
    oracle_boys(Lt, T, F);
    /* level n holds R^n_{tuv} for t+u+v <= Lt-n; start at n = Lt and go down */
    rtab_t *cur = work, *nxt = R0;
    double m2a = -2.0 * alpha;
    /* R^Lt_{000} */
    cur->v[0][0][0] = pow(m2a, Lt) * F[Lt];
    for (int n = Lt - 1; n >= 0; --n) {
        int top = Lt - n;
        /* nxt <- level n from cur (= level n+1) */
        for (int t = 0; t <= top; ++t)
            for (int u = 0; u <= top - t; ++u)
                for (int w = 0; w <= top - t - u; ++w) {
                    double val;
                    if (t == 0 && u == 0 && w == 0) {
                        val = pow(m2a, n) * F[n];
                    } else if (t > 0) {
                        val = L[0] * cur->v[t - 1][u][w];
                        if (t > 1) val += (t - 1) * cur->v[t - 2][u][w];
                    } else if (u > 0) {
                        val = L[1] * cur->v[t][u - 1][w];
                        if (u > 1) val += (u - 1) * cur->v[t][u - 2][w];
                    } else {
                        val = L[2] * cur->v[t][u][w - 1];
                        if (w > 1) val += (w - 1) * cur->v[t][u][w - 2];
                    }
                    nxt->v[t][u][w] = val;
                }
        rtab_t *tmp = cur; cur = nxt; nxt = tmp;
    }
    if (cur != R0) memcpy(R0, cur, sizeof(rtab_t));
}

/* ------------------------------------------------------------------------ */
/* Cartesian components in lexicographic order (x power descending)          */
/* ------------------------------------------------------------------------ */
static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

static void cart_list(int l, int (*c)[3])
{
    int n = 0;
    for (int i = l; i >= 0; --i)
        for (int j = l - i; j >= 0; --j) {
            c[n][0] = i; c[n][1] = j; c[n][2] = l - i - j; ++n;
        }
}

/* ------------------------------------------------------------------------ */
/* One primitive quartet, arbitrary monomial shells la..ld (<= OR_MAXL),     */
/* unnormalised monomials.  out[((ia*nb+ib)*nc+ic)*nd+id]  (eq. eri_formula)  */
/* ------------------------------------------------------------------------ */
typedef struct {
    etab_t Eab[3], Ecd[3];
    rtab_t R0, work;
    double H[2 * OR_MAXL + 2][2 * OR_MAXL + 2][2 * OR_MAXL + 2];
} scratch_t;

/* Two-electron operator: omega = 0 is the Coulomb operator 1/r of eq.
 * eri_formula; omega > 0 is the long-range operator erf(omega r)/r of eq.
 * eri_longrange_definition, whose integrals (eq. eri_longrange_formula) take
 * the prefactor 2 pi^{5/2} omega / (pq sqrt(pq + p omega^2 + q omega^2)) and
 * R^0 at the exponent pq omega^2 / (pq + p omega^2 + q omega^2).  Set before
 * a parallel call and left unchanged during it. */
static double g_omega = 0.0;
void oracle_set_omega(double omega) { g_omega = omega; }
double oracle_get_omega(void) { return g_omega; }

static void prim_block(int la, int lb, int lc, int ld,
                       double a, double b, double c, double d,
                       const double *A, const double *B, const double *C, const double *D,
                       double scale, double *out, scratch_t *S)
{
    double p = a + b, q = c + d;
    double P[3], Q[3], PQ[3];
    for (int k = 0; k < 3; ++k) {
        P[k] = (a * A[k] + b * B[k]) / p;
        Q[k] = (c * C[k] + d * D[k]) / q;
        PQ[k] = P[k] - Q[k];
    }
    double alpha, pref;
    if (g_omega > 0.0) { /* eq. eri_longrange_formula */
        double w2 = g_omega * g_omega, den = p * q + p * w2 + q * w2;
        alpha = p * q * w2 / den;
        pref = scale * 2.0 * pow(OR_PI, 2.5) * g_omega / (p * q * sqrt(den));
    } else {             /* eq. eri_formula */
        alpha = p * q / (p + q);
        pref = scale * 2.0 * pow(OR_PI, 2.5) / (p * q * sqrt(p + q));
    }
    for (int k = 0; k < 3; ++k) {
        e_coeffs(la, lb, a, b, A[k], B[k], S->Eab[k]);
        e_coeffs(lc, ld, c, d, C[k], D[k], S->Ecd[k]);
    }
    int Lt = la + lb + lc + ld;
    r_tensor(Lt, alpha, PQ, &S->R0, &S->work);

    int ca[64][3], cb[64][3], cc[64][3], cd[64][3];
    cart_list(la, ca); cart_list(lb, cb); cart_list(lc, cc); cart_list(ld, cd);
    int na = ncart(la), nb = ncart(lb), nc = ncart(lc), nd = ncart(ld);
    int lab = la + lb;

    for (int ic = 0; ic < nc; ++ic)
        for (int id = 0; id < nd; ++id) {
            const int *k = cc[ic], *l = cd[id];
            /* H[t] = sum_s (-1)^{|s|} E^{kl}_s R_{t+s}, for every bra Hermite t */
            for (int tx = 0; tx <= lab; ++tx)
                for (int ty = 0; ty <= lab - tx; ++ty)
                    for (int tz = 0; tz <= lab - tx - ty; ++tz) {
                        double h = 0.0;
                        for (int sx = 0; sx <= k[0] + l[0]; ++sx)
                            for (int sy = 0; sy <= k[1] + l[1]; ++sy)
                                for (int sz = 0; sz <= k[2] + l[2]; ++sz) {
                                    double e = S->Ecd[0][k[0]][l[0]][sx] *
                                               S->Ecd[1][k[1]][l[1]][sy] *
                                               S->Ecd[2][k[2]][l[2]][sz];
                                    double sg = ((sx + sy + sz) & 1) ? -1.0 : 1.0;
                                    h += sg * e * S->R0.v[tx + sx][ty + sy][tz + sz];
                                }
                        S->H[tx][ty][tz] = h;
                    }
            for (int ia = 0; ia < na; ++ia)
                for (int ib = 0; ib < nb; ++ib) {
                    const int *i = ca[ia], *j = cb[ib];
                    double v = 0.0;
                    for (int tx = 0; tx <= i[0] + j[0]; ++tx)
                        for (int ty = 0; ty <= i[1] + j[1]; ++ty)
                            for (int tz = 0; tz <= i[2] + j[2]; ++tz)
                                v += S->Eab[0][i[0]][j[0]][tx] * S->Eab[1][i[1]][j[1]][ty] *
                                     S->Eab[2][i[2]][j[2]][tz] * S->H[tx][ty][tz];
                    out[((ia * nb + ib) * nc + ic) * nd + id] += pref * v;
                }
        }
}

/* ------------------------------------------------------------------------ */
/* Basis description handed in from Python                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t nshell, natom;
    const int32_t *atom, *l, *nprim, *off; /* per shell */
    const double *exps, *coefs;            /* per primitive; coefs are fully normalised */
    const double *xyz;                     /* [natom][3] */
    const double *qprim;                   /* [nprim_tot][nprim_tot] primitive-pair bounds or NULL */
    int32_t nprim_tot;
    double tau_prim;                       /* primitive quartet kept iff q_ij q_kl >= tau_prim */
} basis_t;

static basis_t mkbasis(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l,
                       const int32_t *nprim, const int32_t *off, const double *exps,
                       const double *coefs, const double *xyz)
{
    basis_t B = {nshell, natom, atom, l, nprim, off, exps, coefs, xyz, NULL, 0, 0.0};
    return B;
}

/* Contracted Cartesian block (ab|cd); shell angular momenta may be overridden
 * (lx >= 0) and a derivative on one centre requested (dcen 0..3, dax 0..2;
 * dcen < 0: plain block).  out is zeroed here. */
static void shell_block(const basis_t *B, int sa, int sb, int sc, int sd,
                        int dcen, int dax, double *out, scratch_t *S)
{
    int sh[4] = {sa, sb, sc, sd};
    int L[4];
    const double *X[4];
    for (int k = 0; k < 4; ++k) {
        L[k] = B->l[sh[k]];
        X[k] = B->xyz + 3 * B->atom[sh[k]];
    }
    int n[4];
    for (int k = 0; k < 4; ++k) n[k] = ncart(L[k]);
    int ntot = n[0] * n[1] * n[2] * n[3];
    memset(out, 0, sizeof(double) * ntot);

    /* derivative path: shifted blocks accumulated into component slots */
    double *tmp = NULL;
    int Lp[4] = {L[0], L[1], L[2], L[3]};
    int np[4] = {n[0], n[1], n[2], n[3]};
    int cl[4][64][3];
    for (int k = 0; k < 4; ++k) cart_list(L[k], cl[k]);
    int clp[64][3], clm[64][3];
    if (dcen >= 0) {
        Lp[dcen] = L[dcen] + 1;
        np[dcen] = ncart(Lp[dcen]);
        cart_list(Lp[dcen], clp);
        if (L[dcen] > 0) cart_list(L[dcen] - 1, clm);
        tmp = (double *)malloc(sizeof(double) * np[0] * np[1] * np[2] * np[3]);
    }

    for (int i0 = 0; i0 < B->nprim[sa]; ++i0)
        for (int i1 = 0; i1 < B->nprim[sb]; ++i1)
            for (int i2 = 0; i2 < B->nprim[sc]; ++i2)
                for (int i3 = 0; i3 < B->nprim[sd]; ++i3) {
                    int pi[4] = {B->off[sa] + i0, B->off[sb] + i1, B->off[sc] + i2, B->off[sd] + i3};
                    /* primitive-pair screening (pGTO pairs, section "Data structure") */
                    if (B->qprim && B->qprim[(size_t)pi[0] * B->nprim_tot + pi[1]] *
                                        B->qprim[(size_t)pi[2] * B->nprim_tot + pi[3]] < B->tau_prim)
                        continue;
                    double e[4], cf = 1.0;
                    for (int k = 0; k < 4; ++k) { e[k] = B->exps[pi[k]]; cf *= B->coefs[pi[k]]; }
                    if (dcen < 0) {
                        prim_block(L[0], L[1], L[2], L[3], e[0], e[1], e[2], e[3],
                                   X[0], X[1], X[2], X[3], cf, out, S);
                        continue;
                    }
                    /* + 2 e (x-A)^{i+1}: block with l+1 on centre dcen */
                    int nn = np[0] * np[1] * np[2] * np[3];
                    memset(tmp, 0, sizeof(double) * nn);
                    prim_block(Lp[0], Lp[1], Lp[2], Lp[3], e[0], e[1], e[2], e[3],
                               X[0], X[1], X[2], X[3], cf * 2.0 * e[dcen], tmp, S);
                    /* scatter: component c of shell dcen gets up-shift slot c+1_ax */
                    for (int a0 = 0; a0 < n[0]; ++a0)
                        for (int a1 = 0; a1 < n[1]; ++a1)
                            for (int a2 = 0; a2 < n[2]; ++a2)
                                for (int a3 = 0; a3 < n[3]; ++a3) {
                                    int idx[4] = {a0, a1, a2, a3};
                                    int cc3[3];
                                    for (int k = 0; k < 3; ++k) cc3[k] = cl[dcen][idx[dcen]][k];
                                    cc3[dax] += 1;
                                    int slot = -1;
                                    for (int s = 0; s < np[dcen]; ++s)
                                        if (clp[s][0] == cc3[0] && clp[s][1] == cc3[1] && clp[s][2] == cc3[2]) slot = s;
                                    int j[4] = {a0, a1, a2, a3};
                                    j[dcen] = slot;
                                    out[((a0 * n[1] + a1) * n[2] + a2) * n[3] + a3] +=
                                        tmp[((j[0] * np[1] + j[1]) * np[2] + j[2]) * np[3] + j[3]];
                                }
                    /* - i_ax (x-A)^{i-1}: block with l-1 on centre dcen */
                    if (L[dcen] > 0) {
                        int Lm[4] = {L[0], L[1], L[2], L[3]};
                        Lm[dcen] -= 1;
                        int nm[4] = {n[0], n[1], n[2], n[3]};
                        nm[dcen] = ncart(Lm[dcen]);
                        int nnm = nm[0] * nm[1] * nm[2] * nm[3];
                        memset(tmp, 0, sizeof(double) * nnm);
                        prim_block(Lm[0], Lm[1], Lm[2], Lm[3], e[0], e[1], e[2], e[3],
                                   X[0], X[1], X[2], X[3], cf, tmp, S);
                        for (int a0 = 0; a0 < n[0]; ++a0)
                            for (int a1 = 0; a1 < n[1]; ++a1)
                                for (int a2 = 0; a2 < n[2]; ++a2)
                                    for (int a3 = 0; a3 < n[3]; ++a3) {
                                        int idx[4] = {a0, a1, a2, a3};
                                        int cc3[3];
                                        for (int k = 0; k < 3; ++k) cc3[k] = cl[dcen][idx[dcen]][k];
                                        int pw = cc3[dax];
                                        if (pw == 0) continue;
                                        cc3[dax] -= 1;
                                        int slot = -1;
                                        for (int s = 0; s < nm[dcen]; ++s)
                                            if (clm[s][0] == cc3[0] && clm[s][1] == cc3[1] && clm[s][2] == cc3[2]) slot = s;
                                        int j[4] = {a0, a1, a2, a3};
                                        j[dcen] = slot;
                                        out[((a0 * n[1] + a1) * n[2] + a2) * n[3] + a3] -=
                                            pw * tmp[((j[0] * nm[1] + j[1]) * nm[2] + j[2]) * nm[3] + j[3]];
                                    }
                    }
                }
    free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Exported helpers                                                          */
/* ------------------------------------------------------------------------ */

/* One primitive block for arbitrary monomial shells (used by the pins). */
void oracle_prim_block(int la, int lb, int lc, int ld, const double *exps4,
                       const double *centres12, double *out)
{
    scratch_t *S = (scratch_t *)malloc(sizeof(scratch_t));
    int n = ncart(la) * ncart(lb) * ncart(lc) * ncart(ld);
    memset(out, 0, sizeof(double) * n);
    prim_block(la, lb, lc, ld, exps4[0], exps4[1], exps4[2], exps4[3],
               centres12, centres12 + 3, centres12 + 6, centres12 + 9, 1.0, out, S);
    free(S);
}

/* One Hermite coefficient table (pins for eq. E_recursion). */
void oracle_e_coeffs(int la, int lb, double a, double b, double Ax, double Bx, double *out)
{
    etab_t E;
    e_coeffs(la, lb, a, b, Ax, Bx, E);
    for (int i = 0; i <= la; ++i)
        for (int j = 0; j <= lb; ++j)
            for (int t = 0; t <= la + lb; ++t)
                out[(i * (lb + 1) + j) * (la + lb + 1) + t] = (t <= i + j) ? E[i][j][t] : 0.0;
}

/* R^0_{tuv} table, dense [Lt+1]^3 (pins for eq. R_recursion). */
void oracle_r_tensor(int Lt, double alpha, const double *L, double *out)
{
    rtab_t *R = (rtab_t *)malloc(sizeof(rtab_t)), *W = (rtab_t *)malloc(sizeof(rtab_t));
    r_tensor(Lt, alpha, L, R, W);
    int n = Lt + 1;
    for (int t = 0; t < n; ++t)
        for (int u = 0; u < n; ++u)
            for (int w = 0; w < n; ++w)
                out[(t * n + u) * n + w] = (t + u + w <= Lt) ? R->v[t][u][w] : 0.0;
    free(R); free(W);
}

/* Contracted Cartesian block of one shell quartet (dcen < 0: no derivative). */
void oracle_shell_block(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l,
                        const int32_t *nprim, const int32_t *off, const double *exps,
                        const double *coefs, const double *xyz,
                        int sa, int sb, int sc, int sd, int dcen, int dax, double *out)
{
    basis_t B = mkbasis(nshell, natom, atom, l, nprim, off, exps, coefs, xyz);
    scratch_t *S = (scratch_t *)malloc(sizeof(scratch_t));
    shell_block(&B, sa, sb, sc, sd, dcen, dax, out, S);
    free(S);
}

/* Schwarz factors Q_ab = sqrt(max_{mu in a, nu in b} |(mu nu|mu nu)|), all pairs. */
void oracle_schwarz(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l,
                    const int32_t *nprim, const int32_t *off, const double *exps,
                    const double *coefs, const double *xyz, double *Q)
{
    basis_t B = mkbasis(nshell, natom, atom, l, nprim, off, exps, coefs, xyz);
#pragma omp parallel
    {
        scratch_t *S = (scratch_t *)malloc(sizeof(scratch_t));
        double *blk = (double *)malloc(sizeof(double) * 10000);
#pragma omp for schedule(dynamic, 4)
        for (int a = 0; a < nshell; ++a)
            for (int b = 0; b <= a; ++b) {
                shell_block(&B, a, b, a, b, -1, 0, blk, S);
                int na = ncart(l[a]), nb = ncart(l[b]);
                double mx = 0.0;
                for (int i = 0; i < na; ++i)
                    for (int j = 0; j < nb; ++j) {
                        double v = fabs(blk[((i * nb + j) * na + i) * nb + j]);
                        if (v > mx) mx = v;
                    }
                Q[a * nshell + b] = Q[b * nshell + a] = sqrt(mx);
            }
        free(blk); free(S);
    }
}

/* Primitive-pair bounds q_ij = |C_i C_j| sqrt(max_c |(ij|ij)_c|) for every pair
 * of primitives (any two shells), [nprim_tot][nprim_tot]. */
void oracle_prim_bounds(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l,
                        const int32_t *nprim, const int32_t *off, const double *exps,
                        const double *coefs, const double *xyz, double *qout)
{
    int32_t ntot = 0;
    for (int s = 0; s < nshell; ++s) ntot += nprim[s];
#pragma omp parallel
    {
        scratch_t *S = (scratch_t *)malloc(sizeof(scratch_t));
        double *blk = (double *)malloc(sizeof(double) * 10000);
#pragma omp for schedule(dynamic, 4)
        for (int a = 0; a < nshell; ++a)
            for (int b = 0; b < nshell; ++b) {
                int na = ncart(l[a]), nb = ncart(l[b]);
                for (int i = 0; i < nprim[a]; ++i)
                    for (int j = 0; j < nprim[b]; ++j) {
                        int pa = off[a] + i, pb = off[b] + j;
                        const double *A = xyz + 3 * atom[a], *Bc = xyz + 3 * atom[b];
                        memset(blk, 0, sizeof(double) * na * nb * na * nb);
                        prim_block(l[a], l[b], l[a], l[b], exps[pa], exps[pb], exps[pa], exps[pb],
                                   A, Bc, A, Bc, 1.0, blk, S);
                        double mx = 0.0;
                        for (int u = 0; u < na; ++u)
                            for (int v = 0; v < nb; ++v) {
                                double x = fabs(blk[((u * nb + v) * na + u) * nb + v]);
                                if (x > mx) mx = x;
                            }
                        qout[(size_t)pa * ntot + pb] = fabs(coefs[pa] * coefs[pb]) * sqrt(mx);
                    }
            }
        free(blk); free(S);
    }
}

/* ------------------------------------------------------------------------ */
/* Point-charge potential (nuclear attraction and QM/MM charges):            */
/* V_mn = sum_C q_C int m(r) n(r) / |r - C| (eqs. v1e_definition,            */
/* v1e_summation_over_C), by eq. v1e_formula:                                */
/*   V_mnC = q_C C_m C_n (2 pi/p) sum_t E^{mn}_t R^0_t(p, P - C).            */
/* ------------------------------------------------------------------------ */

/* Cartesian block of one primitive pair summed over the charges (chg[4k..4k+3]
 * = x, y, z, q), times scale, added to out[ia*nb+ib].  dcharge >= 0: instead
 * the derivative with respect to the position of charge dcharge along axis dax,
 * d/dC_x R^0_{tuv}(p, P - C) = -R^0_{t+1,u,v} (SI eq. si_v1e_derivative_C). */
static void prim_vblock(int la, int lb, double a, double b, const double *A, const double *B,
                        int ncharge, const double *chg, int dcharge, int dax, double scale,
                        double *out, scratch_t *S)
{
    double p = a + b, P[3];
    for (int k = 0; k < 3; ++k) {
        P[k] = (a * A[k] + b * B[k]) / p;
        e_coeffs(la, lb, a, b, A[k], B[k], S->Eab[k]);
    }
    int ca[64][3], cb[64][3];
    cart_list(la, ca);
    cart_list(lb, cb);
    int na = ncart(la), nb = ncart(lb);
    int c0 = dcharge >= 0 ? dcharge : 0, c1 = dcharge >= 0 ? dcharge + 1 : ncharge;
    int Lt = la + lb + (dcharge >= 0 ? 1 : 0);
    for (int c = c0; c < c1; ++c) {
        const double *C = chg + 4 * c;
        double PC[3] = {P[0] - C[0], P[1] - C[1], P[2] - C[2]};
        r_tensor(Lt, p, PC, &S->R0, &S->work);
        double pref = scale * C[3] * 2.0 * OR_PI / p;
        int sh[3] = {0, 0, 0};
        if (dcharge >= 0) {
            sh[dax] = 1;
            pref = -pref;
        }
        for (int ia = 0; ia < na; ++ia)
            for (int ib = 0; ib < nb; ++ib) {
                const int *i = ca[ia], *j = cb[ib];
                double v = 0.0;
                for (int tx = 0; tx <= i[0] + j[0]; ++tx)
                    for (int ty = 0; ty <= i[1] + j[1]; ++ty)
                        for (int tz = 0; tz <= i[2] + j[2]; ++tz)
                            v += S->Eab[0][i[0]][j[0]][tx] * S->Eab[1][i[1]][j[1]][ty] *
                                 S->Eab[2][i[2]][j[2]][tz] * S->R0.v[tx + sh[0]][ty + sh[1]][tz + sh[2]];
                out[ia * nb + ib] += pref * v;
            }
    }
}

/* Contracted Cartesian block of shells (sa, sb).  dcen 0/1: derivative with
 * respect to the centre of sa / sb along dax, by differentiating the basis
 * function, d/dA_x [(x-A_x)^i e^{-a(x-A_x)^2}] = 2a (x-A_x)^{i+1} e - i (x-A_x)^{i-1} e
 * (every charge); dcen 2: derivative with respect to charge dcharge. */
static void shell_vblock(const basis_t *B, int sa, int sb, int ncharge, const double *chg, int dcen,
                         int dax, int dcharge, double *out, scratch_t *S)
{
    int L[2] = {B->l[sa], B->l[sb]};
    int n[2] = {ncart(L[0]), ncart(L[1])};
    const double *X[2] = {B->xyz + 3 * B->atom[sa], B->xyz + 3 * B->atom[sb]};
    memset(out, 0, sizeof(double) * n[0] * n[1]);
    int cl[2][64][3];
    cart_list(L[0], cl[0]);
    cart_list(L[1], cl[1]);
    double tmp[15 * 15];
    for (int i0 = 0; i0 < B->nprim[sa]; ++i0)
        for (int i1 = 0; i1 < B->nprim[sb]; ++i1) {
            int pi[2] = {B->off[sa] + i0, B->off[sb] + i1};
            double e[2] = {B->exps[pi[0]], B->exps[pi[1]]};
            double cf = B->coefs[pi[0]] * B->coefs[pi[1]];
            if (dcen < 0 || dcen == 2) {
                prim_vblock(L[0], L[1], e[0], e[1], X[0], X[1], ncharge, chg, dcen == 2 ? dcharge : -1, dax, cf,
                            out, S);
                continue;
            }
            /* + 2 e (x-A)^{i+1} */
            int Lp[2] = {L[0], L[1]};
            Lp[dcen] += 1;
            int np[2] = {ncart(Lp[0]), ncart(Lp[1])};
            int clp[64][3];
            cart_list(Lp[dcen], clp);
            memset(tmp, 0, sizeof(double) * np[0] * np[1]);
            prim_vblock(Lp[0], Lp[1], e[0], e[1], X[0], X[1], ncharge, chg, -1, 0, cf * 2.0 * e[dcen], tmp, S);
            for (int a0 = 0; a0 < n[0]; ++a0)
                for (int a1 = 0; a1 < n[1]; ++a1) {
                    int idx[2] = {a0, a1}, cc[3];
                    for (int k = 0; k < 3; ++k) cc[k] = cl[dcen][idx[dcen]][k];
                    cc[dax] += 1;
                    int slot = -1;
                    for (int q = 0; q < np[dcen]; ++q)
                        if (clp[q][0] == cc[0] && clp[q][1] == cc[1] && clp[q][2] == cc[2]) slot = q;
                    int j[2] = {a0, a1};
                    j[dcen] = slot;
                    out[a0 * n[1] + a1] += tmp[j[0] * np[1] + j[1]];
                }
            /* - i (x-A)^{i-1} */
            if (L[dcen] > 0) {
                int Lm[2] = {L[0], L[1]};
                Lm[dcen] -= 1;
                int nm[2] = {ncart(Lm[0]), ncart(Lm[1])};
                int clm[64][3];
                cart_list(Lm[dcen], clm);
                memset(tmp, 0, sizeof(double) * nm[0] * nm[1]);
                prim_vblock(Lm[0], Lm[1], e[0], e[1], X[0], X[1], ncharge, chg, -1, 0, cf, tmp, S);
                for (int a0 = 0; a0 < n[0]; ++a0)
                    for (int a1 = 0; a1 < n[1]; ++a1) {
                        int idx[2] = {a0, a1}, cc[3];
                        for (int k = 0; k < 3; ++k) cc[k] = cl[dcen][idx[dcen]][k];
                        int pw = cc[dax];
                        if (pw == 0) continue;
                        cc[dax] -= 1;
                        int slot = -1;
                        for (int q = 0; q < nm[dcen]; ++q)
                            if (clm[q][0] == cc[0] && clm[q][1] == cc[1] && clm[q][2] == cc[2]) slot = q;
                        int j[2] = {a0, a1};
                        j[dcen] = slot;
                        out[a0 * n[1] + a1] -= pw * tmp[j[0] * nm[1] + j[1]];
                    }
            }
        }
}

/* Spherical (or Cartesian if T == NULL) 2-index block from a Cartesian one. */
static void vblock_sph(int la, int lb, const double *T, const int *Toff, const double *cart, double *sph)
{
    int na = ncart(la), nb = ncart(lb), sa = 2 * la + 1, sb = 2 * lb + 1;
    const double *Ta = T + Toff[la], *Tb = T + Toff[lb];
    for (int i = 0; i < sa; ++i)
        for (int j = 0; j < sb; ++j) {
            double v = 0.0;
            for (int x = 0; x < na; ++x)
                for (int y = 0; y < nb; ++y) v += Ta[i * na + x] * Tb[j * nb + y] * cart[x * nb + y];
            sph[i * sb + j] = v;
        }
}

/* V (spherical, nbf x nbf) over every ordered shell pair. */
void oracle_vmatrix(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l,
                    const int32_t *nprim, const int32_t *off, const double *exps, const double *coefs,
                    const double *xyz, const double *T, const int *Toff, const int32_t *ao_off, int32_t nbf,
                    int32_t ncharge, const double *chg, double *V)
{
    basis_t B = mkbasis(nshell, natom, atom, l, nprim, off, exps, coefs, xyz);
    memset(V, 0, sizeof(double) * nbf * nbf);
#pragma omp parallel
    {
        scratch_t *S = (scratch_t *)malloc(sizeof(scratch_t));
        double blk[256], sph[64];
#pragma omp for schedule(dynamic, 1)
        for (int a = 0; a < nshell; ++a)
            for (int b = 0; b < nshell; ++b) {
                shell_vblock(&B, a, b, ncharge, chg, -1, 0, -1, blk, S);
                vblock_sph(l[a], l[b], T, Toff, blk, sph);
                int sa = 2 * l[a] + 1, sb = 2 * l[b] + 1;
                for (int i = 0; i < sa; ++i)
                    for (int j = 0; j < sb; ++j) V[(ao_off[a] + i) * nbf + ao_off[b] + j] = sph[i * sb + j];
            }
        free(S);
    }
}

/* E_V = sum_mn P_mn V_mn and its derivatives at fixed P: with respect to the
 * atoms carrying the basis functions (gatom[natom][3], every ordered shell
 * pair, both centres) and to the charge positions (gchg[ncharge][3]). */
void oracle_vgrad(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l,
                  const int32_t *nprim, const int32_t *off, const double *exps, const double *coefs,
                  const double *xyz, const double *T, const int *Toff, const int32_t *ao_off, int32_t nbf,
                  int32_t ncharge, const double *chg, const double *P, double *gatom, double *gchg)
{
    basis_t B = mkbasis(nshell, natom, atom, l, nprim, off, exps, coefs, xyz);
    memset(gatom, 0, sizeof(double) * 3 * natom);
    memset(gchg, 0, sizeof(double) * 3 * ncharge);
#pragma omp parallel
    {
        scratch_t *S = (scratch_t *)malloc(sizeof(scratch_t));
        double blk[256], sph[64];
        double *ga = (double *)calloc(3 * natom, sizeof(double));
        double *gc = (double *)calloc(3 * (ncharge > 0 ? ncharge : 1), sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int a = 0; a < nshell; ++a)
            for (int b = 0; b < nshell; ++b) {
                int sa = 2 * l[a] + 1, sb = 2 * l[b] + 1;
                for (int cen = 0; cen < 2; ++cen)
                    for (int ax = 0; ax < 3; ++ax) {
                        shell_vblock(&B, a, b, ncharge, chg, cen, ax, -1, blk, S);
                        vblock_sph(l[a], l[b], T, Toff, blk, sph);
                        double g = 0.0;
                        for (int i = 0; i < sa; ++i)
                            for (int j = 0; j < sb; ++j) g += P[(ao_off[a] + i) * nbf + ao_off[b] + j] * sph[i * sb + j];
                        ga[3 * atom[cen == 0 ? a : b] + ax] += g;
                    }
                for (int c = 0; c < ncharge; ++c)
                    for (int ax = 0; ax < 3; ++ax) {
                        shell_vblock(&B, a, b, ncharge, chg, 2, ax, c, blk, S);
                        vblock_sph(l[a], l[b], T, Toff, blk, sph);
                        double g = 0.0;
                        for (int i = 0; i < sa; ++i)
                            for (int j = 0; j < sb; ++j) g += P[(ao_off[a] + i) * nbf + ao_off[b] + j] * sph[i * sb + j];
                        gc[3 * c + ax] += g;
                    }
            }
#pragma omp critical
        {
            for (int i = 0; i < 3 * natom; ++i) gatom[i] += ga[i];
            for (int i = 0; i < 3 * ncharge; ++i) gchg[i] += gc[i];
        }
        free(ga); free(gc); free(S);
    }
}

/* One primitive Cartesian block of V for the pins (unnormalised monomials). */
void oracle_prim_vblock(int la, int lb, const double *exps2, const double *centres6, int32_t ncharge,
                        const double *chg, double *out)
{
    scratch_t *S = (scratch_t *)malloc(sizeof(scratch_t));
    memset(out, 0, sizeof(double) * ncart(la) * ncart(lb));
    prim_vblock(la, lb, exps2[0], exps2[1], centres6, centres6 + 3, ncharge, chg, -1, 0, 1.0, out, S);
    free(S);
}

/* Transform a Cartesian block to the spherical basis with per-l matrices
 * T_l [2l+1][ncart(l)] (row-major, concatenated for l = 0..3 at Toff[l]). */
static void to_sph(const int *L, const double *T, const int *Toff, const double *cart,
                   double *sph, double *w1)
{
    int nc[4], ns[4];
    for (int k = 0; k < 4; ++k) { nc[k] = ncart(L[k]); ns[k] = 2 * L[k] + 1; }
    /* successive single-index transforms; dims (d0,d1,d2,d3) */
    int dims[4] = {nc[0], nc[1], nc[2], nc[3]};
    const double *src = cart;
    double *bufs[2] = {sph, w1};
    int which = 1;
    for (int k = 0; k < 4; ++k) {
        double *dst = bufs[which];
        const double *Tk = T + Toff[L[k]];
        int pre = 1, post = 1;
        for (int m = 0; m < k; ++m) pre *= dims[m];
        for (int m = k + 1; m < 4; ++m) post *= dims[m];
        for (int x = 0; x < pre; ++x)
            for (int s = 0; s < ns[k]; ++s)
                for (int y = 0; y < post; ++y) {
                    double v = 0.0;
                    for (int c = 0; c < nc[k]; ++c)
                        v += Tk[s * nc[k] + c] * src[(x * nc[k] + c) * post + y];
                    dst[(x * ns[k] + s) * post + y] = v;
                }
        dims[k] = ns[k];
        src = dst;
        which ^= 1;
    }
    /* after 4 transforms the result sits in bufs[0] == sph (k=3 wrote bufs[0]) */
}

/* Direct J and K in the spherical AO basis, plain definition over every
 * ordered shell quartet that passes the Schwarz rule.  P is nbf x nbf.
 * Jout/Kout are (re)written. */
void oracle_jk(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l,
               const int32_t *nprim, const int32_t *off, const double *exps,
               const double *coefs, const double *xyz, const double *T, const int *Toff,
               const int32_t *ao_off, int32_t nbf, const double *P, const double *Q, const double *qprim, int32_t nprim_tot, double tau_prim,
               double tau, int want_j, int want_k, double *Jout, double *Kout)
{
    basis_t B = mkbasis(nshell, natom, atom, l, nprim, off, exps, coefs, xyz);
    B.qprim = qprim; B.nprim_tot = nprim_tot; B.tau_prim = tau_prim;
    memset(Jout, 0, sizeof(double) * nbf * nbf);
    memset(Kout, 0, sizeof(double) * nbf * nbf);
#pragma omp parallel
    {
        scratch_t *S = (scratch_t *)malloc(sizeof(scratch_t));
        double *blk = (double *)malloc(sizeof(double) * 10000);
        double *sph = (double *)malloc(sizeof(double) * 10000);
        double *w1 = (double *)malloc(sizeof(double) * 10000);
        double *Jl = (double *)calloc((size_t)nbf * nbf, sizeof(double));
        double *Kl = (double *)calloc((size_t)nbf * nbf, sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int a = 0; a < nshell; ++a)
            for (int b = 0; b < nshell; ++b)
                for (int c = 0; c < nshell; ++c)
                    for (int d = 0; d < nshell; ++d) {
                        if (Q[a * nshell + b] * Q[c * nshell + d] < tau) continue;
                        int L[4] = {l[a], l[b], l[c], l[d]};
                        shell_block(&B, a, b, c, d, -1, 0, blk, S);
                        to_sph(L, T, Toff, blk, sph, w1);
                        int na = 2 * L[0] + 1, nb = 2 * L[1] + 1, nc = 2 * L[2] + 1, nd = 2 * L[3] + 1;
                        for (int i = 0; i < na; ++i)
                            for (int j = 0; j < nb; ++j)
                                for (int k = 0; k < nc; ++k)
                                    for (int m = 0; m < nd; ++m) {
                                        double v = sph[((i * nb + j) * nc + k) * nd + m];
                                        int mu = ao_off[a] + i, nu = ao_off[b] + j;
                                        int la_ = ao_off[c] + k, si = ao_off[d] + m;
                                        if (want_j) Jl[mu * nbf + nu] += v * P[la_ * nbf + si];
                                        if (want_k) Kl[mu * nbf + la_] += v * P[nu * nbf + si];
                                    }
                    }
#pragma omp critical
        {
            for (size_t i = 0; i < (size_t)nbf * nbf; ++i) { Jout[i] += Jl[i]; Kout[i] += Kl[i]; }
        }
        free(Jl); free(Kl); free(w1); free(sph); free(blk); free(S);
    }
}

/* Sampled blocks of J and K for large systems: J block (a,b) = sum over all
 * ordered (c,d) of (ab|cd) P_cd, K block (a,c) = sum over all ordered (b,d)
 * of (ab|cd) P_bd, in the spherical basis.  Output blocks are packed one after
 * another in the order given (J blocks first, then K blocks). */
void oracle_jk_blocks(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l,
                      const int32_t *nprim, const int32_t *off, const double *exps,
                      const double *coefs, const double *xyz, const double *T, const int *Toff,
                      const int32_t *ao_off, int32_t nbf, const double *P, const double *Q, const double *qprim, int32_t nprim_tot, double tau_prim,
                      double tau, int nj, const int32_t *jpairs, int nk, const int32_t *kpairs,
                      const int64_t *out_off, double *out)
{
    basis_t B = mkbasis(nshell, natom, atom, l, nprim, off, exps, coefs, xyz);
    B.qprim = qprim; B.nprim_tot = nprim_tot; B.tau_prim = tau_prim;
    int ntask = nj + nk;
    for (int t = 0; t < ntask; ++t) {
        int x = (t < nj) ? jpairs[2 * t] : kpairs[2 * (t - nj)];
        int y = (t < nj) ? jpairs[2 * t + 1] : kpairs[2 * (t - nj) + 1];
        int nx = 2 * l[x] + 1, ny = 2 * l[y] + 1;
        double *o = out + out_off[t];
        memset(o, 0, sizeof(double) * nx * ny);
        int isj = t < nj;
#pragma omp parallel
        {
            scratch_t *S = (scratch_t *)malloc(sizeof(scratch_t));
            double *blk = (double *)malloc(sizeof(double) * 10000);
            double *sph = (double *)malloc(sizeof(double) * 10000);
            double *w1 = (double *)malloc(sizeof(double) * 10000);
            double *acc = (double *)calloc(nx * ny, sizeof(double));
#pragma omp for schedule(dynamic, 1)
            for (int u = 0; u < nshell; ++u)
                for (int v = 0; v < nshell; ++v) {
                    /* J: quartet (x y | u v); K: quartet (x u | y v) */
                    int a = x, b = isj ? y : u, c = isj ? u : y, d = v;
                    if (Q[a * nshell + b] * Q[c * nshell + d] < tau) continue;
                    int L[4] = {l[a], l[b], l[c], l[d]};
                    shell_block(&B, a, b, c, d, -1, 0, blk, S);
                    to_sph(L, T, Toff, blk, sph, w1);
                    int na = 2 * L[0] + 1, nb = 2 * L[1] + 1, nc = 2 * L[2] + 1, nd = 2 * L[3] + 1;
                    for (int i = 0; i < na; ++i)
                        for (int j = 0; j < nb; ++j)
                            for (int k = 0; k < nc; ++k)
                                for (int m = 0; m < nd; ++m) {
                                    double val = sph[((i * nb + j) * nc + k) * nd + m];
                                    if (isj)
                                        acc[i * ny + j] += val * P[(ao_off[c] + k) * nbf + ao_off[d] + m];
                                    else
                                        acc[i * ny + k] += val * P[(ao_off[b] + j) * nbf + ao_off[d] + m];
                                }
                }
#pragma omp critical
            for (int i = 0; i < nx * ny; ++i) o[i] += acc[i];
            free(acc); free(w1); free(sph); free(blk); free(S);
        }
    }
}

/* Nuclear gradient of E = 1/2 sum P_mn P_ls (mn|ls) - 1/4 sum P_ml P_ns (mn|ls)
 * at fixed P and fixed screening decisions, summing the derivative of every
 * ordered quartet with respect to all four of its centres (plain derivative,
 * no permutational shortcuts).  If only_atom >= 0, only quartets touching that
 * atom are visited and only its gradient row is meaningful.  grad[natom][3]. */
void oracle_grad(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l,
                 const int32_t *nprim, const int32_t *off, const double *exps,
                 const double *coefs, const double *xyz, const double *T, const int *Toff,
                 const int32_t *ao_off, int32_t nbf, const double *P, const double *Q, const double *qprim, int32_t nprim_tot, double tau_prim,
                 double tau, double wj, double wk, int only_atom, double *grad)
{
    basis_t B = mkbasis(nshell, natom, atom, l, nprim, off, exps, coefs, xyz);
    B.qprim = qprim; B.nprim_tot = nprim_tot; B.tau_prim = tau_prim;
    memset(grad, 0, sizeof(double) * 3 * natom);
#pragma omp parallel
    {
        scratch_t *S = (scratch_t *)malloc(sizeof(scratch_t));
        double *blk = (double *)malloc(sizeof(double) * 10000);
        double *sph = (double *)malloc(sizeof(double) * 10000);
        double *w1 = (double *)malloc(sizeof(double) * 10000);
        double *gl = (double *)calloc(3 * natom, sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int a = 0; a < nshell; ++a)
            for (int b = 0; b < nshell; ++b)
                for (int c = 0; c < nshell; ++c)
                    for (int d = 0; d < nshell; ++d) {
                        if (Q[a * nshell + b] * Q[c * nshell + d] < tau) continue;
                        int sh[4] = {a, b, c, d};
                        if (only_atom >= 0 && atom[a] != only_atom && atom[b] != only_atom &&
                            atom[c] != only_atom && atom[d] != only_atom)
                            continue;
                        int L[4] = {l[a], l[b], l[c], l[d]};
                        int na = 2 * L[0] + 1, nb = 2 * L[1] + 1, nc = 2 * L[2] + 1, nd = 2 * L[3] + 1;
                        for (int cen = 0; cen < 4; ++cen) {
                            int at = atom[sh[cen]];
                            if (only_atom >= 0 && at != only_atom) continue;
                            for (int ax = 0; ax < 3; ++ax) {
                                shell_block(&B, a, b, c, d, cen, ax, blk, S);
                                to_sph(L, T, Toff, blk, sph, w1);
                                double g = 0.0;
                                for (int i = 0; i < na; ++i)
                                    for (int j = 0; j < nb; ++j)
                                        for (int k = 0; k < nc; ++k)
                                            for (int m = 0; m < nd; ++m) {
                                                int mu = ao_off[a] + i, nu = ao_off[b] + j;
                                                int la_ = ao_off[c] + k, si = ao_off[d] + m;
                                                double w = wj * 0.5 * P[mu * nbf + nu] * P[la_ * nbf + si]
                                                         - wk * 0.25 * P[mu * nbf + la_] * P[nu * nbf + si];
                                                g += w * sph[((i * nb + j) * nc + k) * nd + m];
                                            }
                                gl[3 * at + ax] += g;
                            }
                        }
                    }
#pragma omp critical
        for (int i = 0; i < 3 * natom; ++i) grad[i] += gl[i];
        free(gl); free(w1); free(sph); free(blk); free(S);
    }
}

/* Evaluate the spherical blocks of a list of shell quartets (q4[4*i..4*i+3])
 * in parallel; returns the sum of all block elements (a checksum).  Used to
 * time the oracle on a sample of a workload. */
double oracle_quartet_batch(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l,
                            const int32_t *nprim, const int32_t *off, const double *exps,
                            const double *coefs, const double *xyz, const double *T, const int *Toff,
                            const double *qprim, int32_t nprim_tot, double tau_prim,
                            int64_t n, const int32_t *q4)
{
    basis_t B = mkbasis(nshell, natom, atom, l, nprim, off, exps, coefs, xyz);
    B.qprim = qprim; B.nprim_tot = nprim_tot; B.tau_prim = tau_prim;
    double total = 0.0;
#pragma omp parallel reduction(+ : total)
    {
        scratch_t *S = (scratch_t *)malloc(sizeof(scratch_t));
        double *blk = (double *)malloc(sizeof(double) * 10000);
        double *sph = (double *)malloc(sizeof(double) * 10000);
        double *w1 = (double *)malloc(sizeof(double) * 10000);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            const int32_t *q = q4 + 4 * i;
            int L[4] = {l[q[0]], l[q[1]], l[q[2]], l[q[3]]};
            shell_block(&B, q[0], q[1], q[2], q[3], -1, 0, blk, S);
            to_sph(L, T, Toff, blk, sph, w1);
            int nn = (2 * L[0] + 1) * (2 * L[1] + 1) * (2 * L[2] + 1) * (2 * L[3] + 1);
            for (int k = 0; k < nn; ++k) total += sph[k];
        }
        free(w1); free(sph); free(blk); free(S);
    }
    return total;
}

/* Threads of the parallel loops that follow (timing only; the results do
 * not depend on it). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Overlap and kinetic energy (eqs. overlap_definition, overlap_formula,    */
/* kinetic_definition, kinetic_formula): with the one-direction Hermite      */
/* coefficients E (whose E^{00}_0 carries that direction's factor of K_AB)   */
/*   S = C (pi/p)^{3/2} E^x_0 E^y_0 E^z_0,                                   */
/*   T = C (pi/p)^{3/2} sum_k t_k prod_{other} E_0,                          */
/*   t_k = -j(j-1)/2 E^{i,j-2}_0 + (2j+1) b E^{i,j}_0 - 2 b^2 E^{i,j+2}_0.    */
/* ------------------------------------------------------------------------ */
static void prim_stblock(int la, int lb, double a, double b, const double *A, const double *B, double scale,
                         double *S, double *T, scratch_t *W)
{
    double p = a + b;
    for (int k = 0; k < 3; ++k) e_coeffs(la, lb + 2, a, b, A[k], B[k], W->Eab[k]);
    int ca[64][3], cb[64][3];
    cart_list(la, ca);
    cart_list(lb, cb);
    int na = ncart(la), nb = ncart(lb);
    double pref = scale * pow(OR_PI / p, 1.5);
    for (int ia = 0; ia < na; ++ia)
        for (int ib = 0; ib < nb; ++ib) {
            double sk[3], tk[3];
            for (int k = 0; k < 3; ++k) {
                int i = ca[ia][k], j = cb[ib][k];
                sk[k] = W->Eab[k][i][j][0];
                double t = (2 * j + 1) * b * W->Eab[k][i][j][0] - 2.0 * b * b * W->Eab[k][i][j + 2][0];
                if (j >= 2) t -= 0.5 * j * (j - 1) * W->Eab[k][i][j - 2][0];
                tk[k] = t;
            }
            S[ia * nb + ib] += pref * sk[0] * sk[1] * sk[2];
            T[ia * nb + ib] += pref * (tk[0] * sk[1] * sk[2] + sk[0] * tk[1] * sk[2] + sk[0] * sk[1] * tk[2]);
        }
}

/* S and T (spherical, nbf x nbf) over every ordered shell pair. */
void oracle_st(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l, const int32_t *nprim,
               const int32_t *off, const double *exps, const double *coefs, const double *xyz, const double *Tsph,
               const int *Toff, const int32_t *ao_off, int32_t nbf, double *S, double *T)
{
    basis_t B = mkbasis(nshell, natom, atom, l, nprim, off, exps, coefs, xyz);
#pragma omp parallel
    {
        scratch_t *W = (scratch_t *)malloc(sizeof(scratch_t));
        double sb[256], tb[256], sph[64];
#pragma omp for schedule(dynamic, 1)
        for (int a = 0; a < nshell; ++a)
            for (int b = 0; b < nshell; ++b) {
                int n = ncart(l[a]) * ncart(l[b]);
                memset(sb, 0, sizeof(double) * n);
                memset(tb, 0, sizeof(double) * n);
                for (int i = 0; i < nprim[a]; ++i)
                    for (int j = 0; j < nprim[b]; ++j)
                        prim_stblock(l[a], l[b], exps[off[a] + i], exps[off[b] + j], xyz + 3 * atom[a],
                                     xyz + 3 * atom[b], B.coefs[off[a] + i] * B.coefs[off[b] + j], sb, tb, W);
                int na = 2 * l[a] + 1, nb = 2 * l[b] + 1;
                vblock_sph(l[a], l[b], Tsph, Toff, sb, sph);
                for (int x = 0; x < na; ++x)
                    for (int y = 0; y < nb; ++y) S[(ao_off[a] + x) * nbf + ao_off[b] + y] = sph[x * nb + y];
                vblock_sph(l[a], l[b], Tsph, Toff, tb, sph);
                for (int x = 0; x < na; ++x)
                    for (int y = 0; y < nb; ++y) T[(ao_off[a] + x) * nbf + ao_off[b] + y] = sph[x * nb + y];
            }
        free(W);
    }
}

/* One primitive Cartesian S and T block for the pins (unnormalised monomials). */
void oracle_prim_stblock(int la, int lb, const double *exps2, const double *centres6, double *S, double *T)
{
    scratch_t *W = (scratch_t *)malloc(sizeof(scratch_t));
    memset(S, 0, sizeof(double) * ncart(la) * ncart(lb));
    memset(T, 0, sizeof(double) * ncart(la) * ncart(lb));
    prim_stblock(la, lb, exps2[0], exps2[1], centres6, centres6 + 3, 1.0, S, T, W);
    free(W);
}

