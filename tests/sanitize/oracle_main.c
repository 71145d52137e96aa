/* Host-side sanitizer run of the CPU oracle (test infrastructure): built by
 * tests/test_oracle_sanitizers.py with AddressSanitizer and
 * UndefinedBehaviorSanitizer together with oracle/oracle.c, it calls every
 * exported routine on a small basis with shells up to f and exits 0 when no
 * error was reported.  The values are not checked here (the pins do that). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_boys(int mmax, double T, double *F);
void oracle_set_omega(double omega);
void oracle_prim_block(int la, int lb, int lc, int ld, const double *exps4, const double *centres12, double *out);
void oracle_e_coeffs(int la, int lb, double a, double b, double Ax, double Bx, double *out);
void oracle_r_tensor(int Lt, double alpha, const double *L, double *out);
void oracle_schwarz(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l, const int32_t *nprim,
                    const int32_t *off, const double *exps, const double *coefs, const double *xyz, double *Q);
void oracle_prim_bounds(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l, const int32_t *nprim,
                        const int32_t *off, const double *exps, const double *coefs, const double *xyz,
                        double *qout);
void oracle_jk(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l, const int32_t *nprim,
               const int32_t *off, const double *exps, const double *coefs, const double *xyz, const double *T,
               const int *Toff, const int32_t *ao_off, int32_t nbf, const double *P, const double *Q,
               const double *qprim, int32_t nprim_tot, double tau_prim, double tau, int want_j, int want_k,
               double *Jout, double *Kout);
void oracle_grad(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l, const int32_t *nprim,
                 const int32_t *off, const double *exps, const double *coefs, const double *xyz, const double *T,
                 const int *Toff, const int32_t *ao_off, int32_t nbf, const double *P, const double *Q,
                 const double *qprim, int32_t nprim_tot, double tau_prim, double tau, double wj, double wk,
                 int only_atom, double *grad);
void oracle_vmatrix(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l, const int32_t *nprim,
                    const int32_t *off, const double *exps, const double *coefs, const double *xyz, const double *T,
                    const int *Toff, const int32_t *ao_off, int32_t nbf, int32_t ncharge, const double *chg,
                    double *V);
void oracle_vgrad(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l, const int32_t *nprim,
                  const int32_t *off, const double *exps, const double *coefs, const double *xyz, const double *T,
                  const int *Toff, const int32_t *ao_off, int32_t nbf, int32_t ncharge, const double *chg,
                  const double *P, double *gatom, double *gchg);
void oracle_st(int32_t nshell, int32_t natom, const int32_t *atom, const int32_t *l, const int32_t *nprim,
               const int32_t *off, const double *exps, const double *coefs, const double *xyz, const double *Tsph,
               const int *Toff, const int32_t *ao_off, int32_t nbf, double *S, double *T);
void oracle_prim_vblock(int la, int lb, const double *exps2, const double *centres6, int32_t ncharge,
                        const double *chg, double *out);
void oracle_prim_stblock(int la, int lb, const double *exps2, const double *centres6, double *S, double *T);

static double urand(unsigned *s)
{
    *s = *s * 1103515245u + 12345u;
    return ((*s >> 8) & 0xffffff) / (double)0x1000000;
}

int main(void)
{
    unsigned seed = 7;
    double F[32], E[2000], R[20 * 20 * 20], blk[10000], L3[3] = {0.3, -0.2, 0.5};
    for (int m = 0; m <= 20; ++m)
        for (int k = 0; k < 12; ++k) oracle_boys(m, 0.0 + 7.5 * k, F);
    for (int la = 0; la <= 4; ++la)
        for (int lb = 0; lb <= 4; ++lb) oracle_e_coeffs(la, lb, 0.7, 1.3, 0.1, -0.4, E);
    for (int Lt = 0; Lt <= 16; ++Lt) oracle_r_tensor(Lt, 0.9, L3, R);
    double ex4[4] = {1.1, 0.6, 2.3, 0.4}, cen[12];
    for (int k = 0; k < 12; ++k) cen[k] = urand(&seed) - 0.5;
    for (int la = 0; la <= 3; ++la)
        for (int lb = 0; lb <= 3; ++lb) {
            oracle_prim_block(la, lb, 3 - la, lb, ex4, cen, blk);
            double chg[8] = {0.2, 0.1, -0.3, -1.0, 1.5, -0.7, 0.4, 0.5};
            oracle_prim_vblock(la, lb, ex4, cen, 2, chg, blk);
            oracle_prim_stblock(la, lb, ex4, cen, blk, blk + 200);
        }
    /* two atoms, shells s(2) p(1) d(1) f(1) on each */
    enum { NSH = 8, NAT = 2 };
    int32_t atom[NSH], l[NSH], nprim[NSH], off[NSH], ao[NSH];
    double exps[16], coefs[16], xyz[6] = {0.0, 0.0, 0.0, 0.9, -0.4, 0.6};
    int32_t np = 0, nbf = 0;
    for (int s = 0; s < NSH; ++s) {
        atom[s] = s / 4;
        l[s] = s % 4;
        nprim[s] = l[s] == 0 ? 2 : 1;
        off[s] = np;
        ao[s] = nbf;
        for (int k = 0; k < nprim[s]; ++k) {
            exps[np] = 0.3 + 2.0 * urand(&seed);
            coefs[np] = 0.2 + urand(&seed);
            ++np;
        }
        nbf += 2 * l[s] + 1;
    }
    /* spherical transforms of l = 0..4 (values arbitrary, sizes as the oracle reads them) */
    int Toff[5];
    double T[245];
    for (int k = 0, o = 0; k <= 4; ++k) {
        Toff[k] = o;
        o += (2 * k + 1) * ((k + 1) * (k + 2) / 2);
    }
    for (int k = 0; k < 245; ++k) T[k] = urand(&seed) - 0.5;
    double *P = calloc((size_t)nbf * nbf, sizeof(double)), *J = calloc((size_t)nbf * nbf, sizeof(double));
    double *K = calloc((size_t)nbf * nbf, sizeof(double)), Q[NSH * NSH], *qp = calloc((size_t)np * np, sizeof(double));
    for (int i = 0; i < nbf; ++i)
        for (int j = 0; j <= i; ++j) P[i * nbf + j] = P[j * nbf + i] = urand(&seed) - 0.5;
    oracle_schwarz(NSH, NAT, atom, l, nprim, off, exps, coefs, xyz, Q);
    oracle_prim_bounds(NSH, NAT, atom, l, nprim, off, exps, coefs, xyz, qp);
    oracle_jk(NSH, NAT, atom, l, nprim, off, exps, coefs, xyz, T, Toff, ao, nbf, P, Q, qp, np, 1e-14, 1e-12, 1, 1,
              J, K);
    oracle_set_omega(0.8);
    oracle_jk(NSH, NAT, atom, l, nprim, off, exps, coefs, xyz, T, Toff, ao, nbf, P, Q, NULL, 0, 0.0, 0.0, 1, 1, J, K);
    oracle_set_omega(0.0);
    double g[3 * NAT], gc[3 * 3];
    oracle_grad(NSH, NAT, atom, l, nprim, off, exps, coefs, xyz, T, Toff, ao, nbf, P, Q, qp, np, 1e-14, 1e-12, 0.5,
                -0.25, -1, g);
    oracle_grad(NSH, NAT, atom, l, nprim, off, exps, coefs, xyz, T, Toff, ao, nbf, P, Q, NULL, 0, 0.0, 0.0, 0.5,
                -0.25, 1, g);
    double chg[12] = {0.0, 0.0, 0.0, -6.0, 0.9, -0.4, 0.6, -1.0, 3.0, 1.0, -2.0, 0.5};
    oracle_vmatrix(NSH, NAT, atom, l, nprim, off, exps, coefs, xyz, T, Toff, ao, nbf, 3, chg, J);
    oracle_vgrad(NSH, NAT, atom, l, nprim, off, exps, coefs, xyz, T, Toff, ao, nbf, 3, chg, P, g, gc);
    oracle_st(NSH, NAT, atom, l, nprim, off, exps, coefs, xyz, T, Toff, ao, nbf, J, K);
    free(P); free(J); free(K); free(qp);
    printf("oracle sanitizer run: nbf %d, done\n", nbf);
    return 0;
}
