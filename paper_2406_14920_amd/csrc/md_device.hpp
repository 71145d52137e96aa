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
// contraction coefficients are carried by PrimPair::K).
template <int LA, int LB>
struct Etab {
    double e[LA + 1][LB + 1][LA + LB + 1];
};

template <int LA, int LB>
__device__ __forceinline__ void etab_build(double PA, double PB, double o2p, Etab<LA, LB> &E)
{
    E.e[0][0][0] = 1.0;
    static_for<0, LA>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        static_for<0, i + 2>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            double v = 0.0;
            if constexpr (t <= i) v = PA * E.e[i][0][t];
            if constexpr (t > 0) v += o2p * E.e[i][0][t - 1];
            if constexpr (t + 1 <= i) v += (double)(t + 1) * E.e[i][0][t + 1];
            E.e[i + 1][0][t] = v;
        });
    });
    static_for<0, LA + 1>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        static_for<0, LB>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            static_for<0, i + j + 2>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                double v = 0.0;
                if constexpr (t <= i + j) v = PB * E.e[i][j][t];
                if constexpr (t > 0) v += o2p * E.e[i][j][t - 1];
                if constexpr (t + 1 <= i + j) v += (double)(t + 1) * E.e[i][j][t + 1];
                E.e[i][j + 1][t] = v;
            });
        });
    });
}

// R^0_{tuv} for t+u+v <= L in registers.  Fs[m] = pref * (-2 alpha)^m F_m.
template <int L>
__device__ __forceinline__ void r_build(const double *Fs, double X, double Y, double Z, double *R)
{
    double cur[nherm(L)];
    cur[0] = Fs[L];
    static_for<0, L>([&](auto lc) {
        constexpr int n = L - 1 - decltype(lc)::value;  // level being built
        double nxt[nherm(L - n)];
        nxt[0] = Fs[n];
        static_for<1, nherm(L - n)>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            constexpr int t = herm_t(k), u = herm_u(k), v = herm_v(k);
            double val;
            if constexpr (t > 0) {
                val = X * cur[herm_idx(t - 1, u, v)];
                if constexpr (t > 1) val += (double)(t - 1) * cur[herm_idx(t - 2, u, v)];
            } else if constexpr (u > 0) {
                val = Y * cur[herm_idx(t, u - 1, v)];
                if constexpr (u > 1) val += (double)(u - 1) * cur[herm_idx(t, u - 2, v)];
            } else {
                val = Z * cur[herm_idx(t, u, v - 1)];
                if constexpr (v > 1) val += (double)(v - 1) * cur[herm_idx(t, u, v - 2)];
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
template <int L>
__device__ __forceinline__ void quartet_fs(const PrimPair &pb, const PrimPair &pk,
                                           const double *__restrict__ btab, double *Fs,
                                           double &X, double &Y, double &Z)
{
    double p = pb.p, q = pk.p;
    double rpq = 1.0 / (p + q);
    double alpha = p * q * rpq;
    X = pb.P[0] - pk.P[0];
    Y = pb.P[1] - pk.P[1];
    Z = pb.P[2] - pk.P[2];
    double T = alpha * (X * X + Y * Y + Z * Z);
    double F[L + 1];
    boys_all<L>(T, F, btab);
    double pref = kTwoPi52 * pb.K * pk.K / (p * q) * sqrt(rpq);
    double m2a = -2.0 * alpha;
    double s = pref;
#pragma unroll
    for (int m = 0; m <= L; ++m) {
        Fs[m] = s * F[m];
        s *= m2a;
    }
}

}  // namespace md
