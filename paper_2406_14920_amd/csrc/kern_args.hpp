// kern_args.hpp -- argument blocks passed by value to the J/K kernels.
#pragma once
#include <stdint.h>

#include "md_common.hpp"

namespace md {

// One (bra class, ket class) exchange launch over canonical shell quartets
// (ab|cd).  The pairs of each class are held in an exchange view: grouped by
// contraction length (largest first), Q descending inside a group.  The work
// list is a sequence of rows; row r pairs bra rows[r].x with the kets
// rows[r].y, rows[r].y + 1, ... of one contraction group, of which the first
// prefix[r+1]-prefix[r] are visited (those passing the Schwarz rule and, in a
// class with itself, the canonical order).  Rows run group pair by group
// pair, so neighbouring work items have equal contraction lengths.
struct KArgs {
    const CPair *bra;        // exchange view of class X
    const CPair *ket;        // exchange view of class Y
    const int2 *rows;        // [nrows] (bra index, first ket index of the row's group)
    const int64_t *prefix;   // [nrows+1] cumulative ket counts
    int64_t nwork;           // prefix[nrows]
    int32_t nrows;
    int32_t same;            // bra class == ket class: the diagonal quartet (ab|ab) gets 1/2
    const PrimPair *pp;
    const double *boys;
    const double *D;         // Cartesian density, ld x ld
    double *Kacc;            // Cartesian exchange accumulator, ld x ld
    int32_t ld;
    double tau_prim;
    const double *eprod_bra; // Hermite products of class-X primitive pairs
    int32_t pbase_bra;
    const double *eprod_ket; // Hermite products of class-Y primitive pairs
    int32_t pbase_ket;
    // mixed precision: single-precision copies of the products, tile mode
    // (0 all, 1 double-precision tiles, 2 single-precision tiles), threshold,
    // contracted Q of both classes and the shell-pair density bounds (nsh x nsh)
    const float *eprodf_bra;
    const float *eprodf_ket;
    int32_t mode;
    double tau_mix;
    const double *Qbra, *Qket;  // Q in exchange-view order
    const double *Pm;
    int32_t nsh;
    int32_t grid_cap;        // workgroups of a range-walking launch (0: default)
    double om2;              // omega^2 of the operator erf(omega r)/r; 0: 1/r
    // > 0: a quartet whose density-weighted bound Q_ab Q_cd max|D| (the four
    // blocks its digestion reads) is below tau_dens is skipped (Qbra, Qket,
    // Pm, nsh set)
    double tau_dens;
    // 0: kets grouped by their first shell c (the items of a row share the
    // K_ac, K_bc targets, which are summed across lanes first); 1: grouped by
    // the second shell d (K_ad, K_bd shared).  Lane-per-item kernels only.
    int32_t inv;
};

// The rows of an exchange work list run bra by bra and, inside a bra, group
// by group: the items of one row share the bra (ab| and the ket shell c, so
// their K_ac and K_bc contributions go to the same elements.
// Row r of an exchange work list: bra pair, first ket index and ket count.
struct KRow {
    int ib, kb, cnt;
};
__device__ __forceinline__ KRow k_row(const int2 *rows, const int64_t *prefix, int r)
{
    const int2 v = rows[r];
    return KRow{v.x, v.y, (int)(prefix[r + 1] - prefix[r])};
}
// row holding work item w (prefix ascending, prefix[0] = 0)
__device__ __forceinline__ int k_find_row(const int64_t *prefix, int nrows, int64_t w)
{
    int lo = 0, hi = nrows;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= w) lo = mid; else hi = mid;
    }
    return lo;
}
// Segmented sums over a wavefront.  The lanes that share a key (the work-list
// row: one bra and one ket shell c) are contiguous; seg_links gives, per
// doubling step k, whether lane + 2^k holds the same key, and seg_sum then
// leaves in the first lane of every run the sum over the run (a downward
// Hillis-Steele scan cut at key changes).  Every lane of the wavefront must
// take part.
struct SegLinks {
    uint32_t same;  // bit k: lane + 2^k is in this lane's run
    bool head;      // first lane of its run
};
__device__ __forceinline__ SegLinks seg_links(int key)
{
    const int lane = threadIdx.x & 63;
    SegLinks L{0u, true};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int off = 1 << k;
        const int ko = __shfl_down(key, off);
        if (lane + off < 64 && ko == key) L.same |= 1u << k;
    }
    const int kp = __shfl_up(key, 1);
    L.head = lane == 0 || kp != key;
    return L;
}
__device__ __forceinline__ double seg_sum(double v, const SegLinks &L)
{
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double o = __shfl_down(v, 1 << k);
        if (L.same & (1u << k)) v += o;
    }
    return v;
}

// the diagonal quartet (ab|ab) of a class with itself
__device__ __forceinline__ bool same_pair(const CPair &A, const CPair &B)
{
    return A.sh1 == B.sh1 && A.sh2 == B.sh2;
}

// J-engine launch: bra primitive pairs of class X against ket contracted
// pairs [j0, j1) of class Y.
struct JArgs {
    const PrimPair *pp;
    const int32_t *owner;    // contracted pair (index inside class X) of each bra primitive pair
    const double *Qbra;      // Q of class-X contracted pairs
    int32_t pbase;           // first primitive pair of class X
    int32_t nbp;             // number of class-X primitive pairs
    const CPair *ket;        // class-Y contracted pairs
    const double *Qket;
    int32_t nket;
    int32_t kchunk;          // ket contracted pairs per work item
    const double *Dt;        // Hermite density of class-Y primitive pairs (nherm(LY) each)
    int32_t dt_base;         // primitive pair index that Dt[0] belongs to
    double *Jh;              // Hermite J of class-X primitive pairs (nherm(LX) each)
    const double *boys;
    double tau, tau_prim;
    // mixed precision: single-precision Hermite density, tile mode, threshold
    // and Q_cd max|D_cd| of every class-Y ket pair
    const float *Dtf;
    int32_t mode;
    double tau_mix;
    const double *QDket;
    double om2;              // omega^2 of the operator erf(omega r)/r; 0: 1/r
    // > 0: a ket pair whose Q_ab Q_cd max|D_cd| (Q_ab the wavefront's largest)
    // is below tau_dens is skipped (Qbra, QDket set)
    double tau_dens;
    // > 0: each ket chunk (blockIdx.y) stores its sums with plain stores at
    // Jh + chunk * jh_part (zeros where it has no kets), for a fixed-order
    // reduction over the chunks; 0: atomic additions into Jh
    int64_t jh_part;
};

// Bra-shared exchange launch: one workgroup per chunk of up to 64
// consecutive work items of one bra (rows as in KArgs).
struct KPArgs {
    const CPair *bra;
    const CPair *ket;
    const int4 *chunks;      // (first row, offset of the first item in it, items, rows spanned)
    const int2 *rows;
    const int64_t *prefix;   // cumulative ket counts of the rows
    int32_t same;
    const PrimPair *pp;
    const double *eprod_bra;  // class-X products, pair g at (g - pbase_bra) * SB
    int32_t pbase_bra;
    const double *eprod_ket;
    int32_t pbase_ket;
    const double *boys;
    const double *D;
    double *Kacc;
    int32_t ld;
    double tau_prim;
    const float *eprodf_bra;
    const float *eprodf_ket;
    int32_t mode;
    double tau_mix;
    const double *Qbra, *Qket;
    const double *Pm;
    int32_t nsh;
    double om2;              // omega^2 of the operator erf(omega r)/r; 0: 1/r
    double tau_dens;         // as in KArgs
    int32_t inv;             // as in KArgs
};

// Exchange-gradient launch: the exchange work list plus the per-workgroup
// gradient partials (gridDim.x x natom x 3).
struct KGArgs {
    KArgs k;
    double *partial;
    int32_t natom;
};

// Coulomb-gradient contraction over the contracted pairs of one class.
struct JGArgs {
    const CPair *cp;
    int32_t ncp;
    const PrimPair *pp;
    const double *Jh1;   // Hermite J of order LX+1 of every class-X primitive pair
    int32_t jh_base;     // primitive pair index that Jh1[0] belongs to
    const double *D;     // Cartesian density
    int32_t ld;
    double *pg;          // [ncp][6]: dE_J/dA, dE_J/dB of each contracted pair
};

}  // namespace md
