// launch.hpp -- host-side entry points of the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "kern_args.hpp"

namespace md {

struct ShellMap {
    const int32_t *shell_of_cart;
    const int32_t *shell_of_sph;
    const int32_t *l;
    const int32_t *cart_off;
    const int32_t *sph_off;
};

bool launch_k_pair_0(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, hipStream_t st);
bool launch_k_pair_1(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, hipStream_t st);
bool launch_k_pair_2(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, hipStream_t st);
bool launch_k_pair_3(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, hipStream_t st);
bool launch_k_pair_4(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, hipStream_t st);
bool launch_k_pair_5(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, hipStream_t st);
bool launch_k_pair_6(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, hipStream_t st);
bool launch_k_pair_7(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, hipStream_t st);
void launch_eprod(int la, int lb, const PrimPair *pp, int pbase, int n, double *out, hipStream_t st);
int eprod_size(int la, int lb);
bool launch_k_small(int la, int lb, int lc, int ld, const KArgs &a, hipStream_t st);
bool launch_k_wave_0(int la, int lb, int lc, int ld, const KArgs &a, hipStream_t st);
bool launch_k_wave_1(int la, int lb, int lc, int ld, const KArgs &a, hipStream_t st);
bool launch_k_wave_2(int la, int lb, int lc, int ld, const KArgs &a, hipStream_t st);
bool launch_k_wave_3(int la, int lb, int lc, int ld, const KArgs &a, hipStream_t st);
bool launch_k_wave_4(int la, int lb, int lc, int ld, const KArgs &a, hipStream_t st);
bool launch_k_wave_5(int la, int lb, int lc, int ld, const KArgs &a, hipStream_t st);

void launch_hermite_density(int lc, int ld, const CPair *cp, int ncp, const PrimPair *pp,
                            const double *D, int ldd, double *Dt, int dt_base, hipStream_t st);
void launch_hermite_to_cart(int la, int lb, const CPair *cp, int ncp, const PrimPair *pp,
                            const double *Jh, int jh_base, double *Jacc, int ld, hipStream_t st);
bool launch_jeng(int lx, int ly, const JArgs &a, hipStream_t st);

void launch_schwarz(int la, int lb, const CPair *cp, int ncp, PrimPair *pp, double *Q,
                    const double *boys, hipStream_t st);
void launch_p_to_cart(const double *P, int nbf, double *Pc, int nc, const ShellMap &m, int sph,
                      hipStream_t st);
void launch_acc_to_out(const double *Acc, int nc, double *Out, int nbf, const ShellMap &m, int sph,
                       hipStream_t st);
void launch_fill_zero(double *x, int64_t n, hipStream_t st);
void launch_k_count(const KArgs &a, unsigned long long *out, hipStream_t st);
void launch_j_count(const JArgs &a, unsigned long long *out, hipStream_t st);

}  // namespace md
