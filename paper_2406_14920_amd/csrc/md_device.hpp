// md_device.hpp -- compile-time McMurchie-Davidson building blocks kept in
// registers: Hermite expansion coefficients (eq. E_recursion), auxiliary
// integrals (eq. R_recursion) and the contraction of eq. eri_formula.
#pragma once
#include <type_traits>

#include "md_common.hpp"

namespace md {

template <int Begin, int End, typename F>
__host__ __device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (Begin < End) {
        f(std::integral_constant<int, Begin>{});
        static_for<Begin + 1, End>(f);
    }
}

// 1D Hermite expansion coefficients E^{ij}_t, i <= LA, j <= LB, t <= i+j, for
// one Cartesian direction; E^{00}_0 = 1 (the Gaussian product prefactor and the
// contraction coefficients are carried by PrimPair::K).  T is the arithmetic
// type of the primitive integrals (double, or float for the single-precision
// share of the mixed mode).
template <int LA, int LB, typename T = double>
struct Etab {
    T e[LA + 1][LB + 1][LA + LB + 1];
};

template <int LA, int LB, typename T>
__device__ __forceinline__ void etab_build(T PA, T PB, T o2p, Etab<LA, LB, T> &E)
{
    E.e[0][0][0] = T(1);
    static_for<0, LA>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        static_for<0, i + 2>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            T v = T(0);
            if constexpr (t <= i) v = PA * E.e[i][0][t];
            if constexpr (t > 0) v += o2p * E.e[i][0][t - 1];
            if constexpr (t + 1 <= i) v += T(t + 1) * E.e[i][0][t + 1];
            E.e[i + 1][0][t] = v;
        });
    });
    static_for<0, LA + 1>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        static_for<0, LB>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            static_for<0, i + j + 2>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                T v = T(0);
                if constexpr (t <= i + j) v = PB * E.e[i][j][t];
                if constexpr (t > 0) v += o2p * E.e[i][j][t - 1];
                if constexpr (t + 1 <= i + j) v += T(t + 1) * E.e[i][j][t + 1];
                E.e[i][j + 1][t] = v;
            });
        });
    });
}

// R^0_{tuv} for t+u+v <= L in registers.  Fs[m] = pref * (-2 alpha)^m F_m.
template <int L, typename T>
__device__ __forceinline__ void r_build(const T *Fs, T X, T Y, T Z, T *R)
{
    T cur[nherm(L)];
    cur[0] = Fs[L];
    static_for<0, L>([&](auto lc) {
        constexpr int n = L - 1 - decltype(lc)::value;  // level being built
        T nxt[nherm(L - n)];
        nxt[0] = Fs[n];
        static_for<1, nherm(L - n)>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            constexpr int t = herm_t(k), u = herm_u(k), v = herm_v(k);
            T val;
            if constexpr (t > 0) {
                val = X * cur[herm_idx(t - 1, u, v)];
                if constexpr (t > 1) val += T(t - 1) * cur[herm_idx(t - 2, u, v)];
            } else if constexpr (u > 0) {
                val = Y * cur[herm_idx(t, u - 1, v)];
                if constexpr (u > 1) val += T(u - 1) * cur[herm_idx(t, u - 2, v)];
            } else {
                val = Z * cur[herm_idx(t, u, v - 1)];
                if constexpr (v > 1) val += T(v - 1) * cur[herm_idx(t, u, v - 2)];
            }
            nxt[k] = val;
        });
        static_for<0, nherm(L - n)>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            cur[k] = nxt[k];
        });
    });
    static_for<0, nherm(L)>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        R[k] = cur[k];
    });
}

// Prefactor and scaled Boys values of one primitive quartet (eq. eri_formula):
// Fs[m] = 2 pi^{5/2}/(pq sqrt(p+q)) K_ab K_cd (-2 alpha)^m F_m(alpha |PQ|^2).
// The Boys values, the prefactor and the powers of -2 alpha are formed in
// double precision whatever T is (their range exceeds single precision for
// tight exponents); only the finished G_m and the separation P - Q are
// rounded to T.
//
// The long-range operator erf(omega r)/r (eq. eri_longrange_formula) takes
// the same form with alpha -> alpha s and the prefactor times sqrt(s),
// s = omega^2 / (alpha + omega^2); om2 = omega^2, 0 for the Coulomb operator.
__device__ __forceinline__ void longrange_scale(double om2, double &alpha, double &pref)
{
    if (om2 > 0.0) {
        const double s = om2 / (alpha + om2);
        alpha *= s;
        pref *= sqrt(s);
    }
}

template <int L, typename T>
__device__ __forceinline__ void quartet_fs(const PrimPair &pb, const PrimPair &pk,
                                           const double *__restrict__ btab, T *Fs, T &X, T &Y, T &Z,
                                           double om2)
{
    double p = pb.p, q = pk.p;
    // 1/sqrt(p+q) once; 1/(pq) from the stored 1/(2p), 1/(2q): no division
    const double rs = rsqrt(p + q);
    const double rpq = rs * rs;
    double alpha = p * q * rpq;
    const double dx = pb.P[0] - pk.P[0];
    const double dy = pb.P[1] - pk.P[1];
    const double dz = pb.P[2] - pk.P[2];
    X = (T)dx;
    Y = (T)dy;
    Z = (T)dz;
    double pref = kTwoPi52 * pb.K * pk.K * (4.0 * pb.o2p * pk.o2p) * rs;
    longrange_scale(om2, alpha, pref);
    double Tb = alpha * (dx * dx + dy * dy + dz * dz);
    double F[L + 1];
    boys_all<L>(Tb, F, btab);
    double m2a = -2.0 * alpha;
    double s = pref;
#pragma unroll
    for (int m = 0; m <= L; ++m) {
        Fs[m] = (T)(s * F[m]);
        s *= m2a;
    }
}

// Single-precision form of eq. eri_formula.  The double-precision quantities
// span far more than the single-precision range for tight shells (K_ab K_cd
// and (2 alpha)^m alone reach 1e30 and beyond), so the single-precision share
// evaluates an exactly rescaled version of the same sums.  With c = sqrt(2p)
// of the bra pair, the closed form of R (see wave_r.hpp) gives
//     R_N(X, G) c^{-|N|} = R_N(c X, G~),   G~_m = G_m / (2p)^m,
// so that
//     (ab|cd) = sum_t [K_ab E^{ab}_t c^{|t|}] sum_s (-1)^{|s|} [K_cd E^{cd}_s c^{|s|}] R~_{t+s}
// with R~ built by the usual recursion from X~ = c (P - Q) and
//     G~_m = 2 pi^{5/2} / (p q sqrt(p+q)) (-q/(p+q))^m F_m,
// every factor of order one.  The ket factor is stored per pair as
// K_cd E^{cd}_s (2q)^{|s|/2} and multiplied by r^{|s|}, r = sqrt(p/q).
// F_m, the powers and the prefactor are formed in double and then rounded.
// Long-range operator: alpha -> alpha s0, w -> w s0, prefactor times
// sqrt(s0), s0 = omega^2/(alpha + omega^2).
template <int L>
__device__ __forceinline__ void quartet_fs_scaled(const PrimPair &pb, const PrimPair &pk,
                                                  const double *__restrict__ btab, float *Fs, float &X,
                                                  float &Y, float &Z, float &r, double om2)
{
    const double p = pb.p, q = pk.p;
    const double rs = rsqrt(p + q);
    const double rpq = rs * rs;
    double alpha = p * q * rpq;
    const double dx = pb.P[0] - pk.P[0];
    const double dy = pb.P[1] - pk.P[1];
    const double dz = pb.P[2] - pk.P[2];
    double s = kTwoPi52 * (4.0 * pb.o2p * pk.o2p) * rs;
    double w = -q * rpq;
    if (om2 > 0.0) {
        const double s0 = om2 / (alpha + om2);
        alpha *= s0;
        w *= s0;
        s *= sqrt(s0);
    }
    double F[L + 1];
    boys_all<L>(alpha * (dx * dx + dy * dy + dz * dz), F, btab);
    const double c = sqrt(2.0 * p);
    X = (float)(c * dx);
    Y = (float)(c * dy);
    Z = (float)(c * dz);
    r = (float)sqrt(p / q);
#pragma unroll
    for (int m = 0; m <= L; ++m) {
        Fs[m] = (float)(s * F[m]);
        s *= w;
    }
}

// Powers x^0..x^N (N compile-time).
template <int N, typename T>
__device__ __forceinline__ void powers(T x, T *pw)
{
    pw[0] = T(1);
#pragma unroll
    for (int k = 1; k <= N; ++k) pw[k] = pw[k - 1] * x;
}

// Scale a 1D Hermite table: E_t *= k c^t.
template <int LA, int LB>
__device__ __forceinline__ void etab_scale(Etab<LA, LB, float> &E, float c, float k)
{
    float w[LA + LB + 1];
    w[0] = k;
#pragma unroll
    for (int t = 1; t <= LA + LB; ++t) w[t] = w[t - 1] * c;
#pragma unroll
    for (int i = 0; i <= LA; ++i)
#pragma unroll
        for (int j = 0; j <= LB; ++j)
#pragma unroll
            for (int t = 0; t <= i + j; ++t) E.e[i][j][t] *= w[t];
}

// Precision of a tile of work in the mixed mode (the paper's rule: a quartet
// is evaluated in double precision when its density-weighted Schwarz bound
// Q_ab Q_cd max|D| reaches the threshold).  A tile is the unit one wavefront
// evaluates together; it runs in double precision if any quartet in it does.
// Mode 0 evaluates every tile (all-double build), mode 1 only the tiles that
// need double precision, mode 2 only the others; launches of modes 1 and 2
// over the same work list with the same geometry partition it exactly.
__device__ __forceinline__ bool mix_take(int mode, bool lane_needs_fp64)
{
    if (mode == 0) return true;
    const bool any = __ballot(lane_needs_fp64 ? 1 : 0) != 0ull;
    return (mode == 1) == any;
}

// Density bound of an exchange quartet (ab|cd): the four density blocks its
// 8-fold digestion reads (D_bd, D_bc, D_ad, D_ac).
__device__ __forceinline__ double k_dens_bound(const double *__restrict__ Pm, int nsh, const CPair &A,
                                               const CPair &B)
{
    const double *ra = Pm + (int64_t)A.sh1 * nsh, *rb = Pm + (int64_t)A.sh2 * nsh;
    return fmax(fmax(ra[B.sh1], ra[B.sh2]), fmax(rb[B.sh1], rb[B.sh2]));
}

template <typename T>
__device__ __forceinline__ const T *pick(const double *d, const float *f)
{
    if constexpr (sizeof(T) == 4) return f; else return d;
}

}  // namespace md
