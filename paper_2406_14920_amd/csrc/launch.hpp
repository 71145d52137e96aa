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

bool launch_k_pair_0(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, bool fp32, hipStream_t st);
bool launch_k_pair_1(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, bool fp32, hipStream_t st);
bool launch_k_pair_2(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, bool fp32, hipStream_t st);
bool launch_k_pair_3(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, bool fp32, hipStream_t st);
bool launch_k_pair_4(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, bool fp32, hipStream_t st);
bool launch_k_pair_5(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, bool fp32, hipStream_t st);
bool launch_k_pair_6(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, bool fp32, hipStream_t st);
bool launch_k_pair_7(int la, int lb, int lc, int ld, const KPArgs &a, int nchunks, bool fp32, hipStream_t st);
void launch_eprod(int la, int lb, const PrimPair *pp, int pbase, int n, double *out, hipStream_t st);
void launch_eprod(int la, int lb, const PrimPair *pp, int pbase, int n, float *out, hipStream_t st);
int eprod_size(int la, int lb);
bool launch_k_small(int la, int lb, int lc, int ld, const KArgs &a, bool fp32, hipStream_t st);
bool launch_k_wave_0(int la, int lb, int lc, int ld, const KArgs &a, bool fp32, hipStream_t st);
bool launch_k_wave_1(int la, int lb, int lc, int ld, const KArgs &a, bool fp32, hipStream_t st);
bool launch_k_wave_2(int la, int lb, int lc, int ld, const KArgs &a, bool fp32, hipStream_t st);
bool launch_k_wave_3(int la, int lb, int lc, int ld, const KArgs &a, bool fp32, hipStream_t st);
bool launch_k_wave_4(int la, int lb, int lc, int ld, const KArgs &a, bool fp32, hipStream_t st);
bool launch_k_wave_5(int la, int lb, int lc, int ld, const KArgs &a, bool fp32, hipStream_t st);

void launch_hermite_density(int lc, int ld, const CPair *cp, int ncp, const PrimPair *pp,
                            const double *D, int ldd, double *Dt, float *Dtf, int dt_base, hipStream_t st);
void launch_hermite_to_cart(int la, int lb, const CPair *cp, int ncp, const PrimPair *pp,
                            const double *Jh, int jh_base, double *Jacc, int ld, hipStream_t st);
bool launch_jeng(int lx, int ly, const JArgs &a, bool fp32, hipStream_t st);
void launch_jh_reduce(const double *part, int nch, int64_t stride, double *out, int64_t n, hipStream_t st);

void launch_schwarz(int la, int lb, const CPair *cp, int ncp, PrimPair *pp, double *Q,
                    const double *boys, hipStream_t st);
void launch_p_to_cart(const double *P, int nbf, double *Pc, int nc, const ShellMap &m, int sph,
                      hipStream_t st);
void launch_acc_to_out(const double *Acc, int nc, double *Out, int nbf, const ShellMap &m, int sph,
                       hipStream_t st);
void launch_fill_zero(double *x, int64_t n, hipStream_t st);
void launch_density_bounds(const double *Pc, int nc, const int32_t *l, const int32_t *coff, int nsh,
                           double *Pm, const CPair *cp, const double *Q, int ncp, double *QD, hipStream_t st);
// primitive quartets (out[0]) and work items (out[1]) of the single-precision
// share of one mixed-precision launch; kind 0 = lane-per-quartet tiles of 64,
// 1 = one quartet per tile, 2 = bra-shared chunks
void launch_k_count_mix(const KArgs &a, int kind, const int4 *chunks, int nchunks, unsigned long long *out,
                        hipStream_t st);
// primitive quartets of the single-precision share of a J-engine launch;
// per_bra = 1 when the tile is a single bra primitive pair
void launch_j_count_mix(const JArgs &a, int per_bra, unsigned long long *out, hipStream_t st);
void launch_k_count(const KArgs &a, unsigned long long *out, hipStream_t st);
void launch_j_count(const JArgs &a, unsigned long long *out, hipStream_t st);

bool launch_kg_0(int la, int lb, int lc, int ld, const KGArgs &g, int blocks, hipStream_t st);
bool launch_kg_1(int la, int lb, int lc, int ld, const KGArgs &g, int blocks, hipStream_t st);
bool launch_kg_2(int la, int lb, int lc, int ld, const KGArgs &g, int blocks, hipStream_t st);
bool launch_kg_3(int la, int lb, int lc, int ld, const KGArgs &g, int blocks, hipStream_t st);
void launch_jgrad(int la, int lb, const JGArgs &g, hipStream_t st);
// Exchange-gradient classes served by the lane-per-quartet kernel kg_small
// (every table in registers); the others use the wavefront kernel kg_wave.
// The larger lane-per-quartet classes spill kilobytes per lane and run
// faster as wavefronts summing over the ket primitive pairs (timed per class).
__host__ __device__ constexpr bool kg_small_class(int la, int lb, int lc, int ld)
{
    return (la == 0 && lb == 0 && lc == 0 && ld == 0) || (la == 1 && lb == 0 && lc == 0 && ld == 0) ||
           (la == 1 && lb == 0 && lc == 1 && ld == 0) || (la == 1 && lb == 1 && lc == 0 && ld == 0) ||
           (la == 1 && lb == 1 && lc == 1 && ld == 0) || (la == 2 && lb == 0 && lc == 0 && ld == 0) ||
           (la == 2 && lb == 0 && lc == 1 && ld == 0) || (la == 2 && lb == 0 && lc == 1 && ld == 1) ||
           (la == 2 && lb == 0 && lc == 2 && ld == 0) || (la == 3 && lb == 0 && lc == 0 && ld == 0);
}

// Fixed-order sum of the exchange partials and Coulomb pair terms into
// grad (natom x 3); part holds grad_reduce_chunks(ncp, nkblocks) x 3 natom
// doubles of scratch.
int grad_reduce_chunks(int ncp, int64_t nkblocks);
void launch_grad_reduce(const CPair *cp, int ncp, const double *pg, const double *kpart, int64_t nkblocks,
                        int natom, double *grad, double *part, hipStream_t st);
void launch_energy(const double *P, const double *J, const double *K, int64_t n2, double *E, hipStream_t st);

// grid.hip: bounding spheres of 64-point blocks; density (and gradient, if
// grad) added into rho/grad; the matrix sums of one pair class
void launch_grid_blocks(const double *pts, int64_t npts, double4 *bsph, hipStream_t st);
void launch_grid_rho(int la, int lb, const CPair *cp, int ncp, const PrimPair *pp, const double4 *psph,
                     const double *xyz, const double *D, int ld, const double *pts, int64_t npts,
                     const double4 *bsph, double *rho, double *grad, hipStream_t st);
void launch_grid_vmat(int la, int lb, const CPair *cp, int ncp, const PrimPair *pp, const double4 *psph,
                      const double *xyz, const double *pts, int64_t npts, const double4 *bsph, const double *v0,
                      const double *v1, double *Vacc, int ld, hipStream_t st);
// overlap and kinetic energy of one pair class into the accumulators (potential.hip)
void launch_st_pair(int la, int lb, const CPair *cp, int ncp, const PrimPair *pp, double *Sacc, double *Tacc, int ld,
                    hipStream_t st);
// point-charge potential (potential.hip); chg holds [n][4] = x, y, z, q
// Hermite potential of order L of npp primitive pairs into Vh [npp][nherm(L)];
// with nsplit > 1 the charges are split over nsplit launches' worth of
// workgroups whose sums go to part [nsplit][npp][nherm(L)] and are reduced in
// order.  potential_splits picks nsplit within cap_doubles of part.
int potential_splits(int npp, int nchg, int L, int64_t cap_doubles);
bool launch_vh(int L, const PrimPair *pp, int pbase, int npp, const double *chg, int nchg, const double *btab,
               double *Vh, double *part, int nsplit, hipStream_t st);
bool launch_vgrad_charge(int L, const PrimPair *pp, int pbase, int npp, const double *Dt, const double *chg,
                         int nchg, const double *btab, double *part, int nshare, double *gchg, hipStream_t st);

}  // namespace md
