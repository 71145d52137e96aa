// jeng_reg.hpp -- J-engine step 2 for high total Hermite order with every
// operand in registers: one lane per bra primitive pair, kets wave-uniform.
// R^0_N is never stored: each entry is formed from the closed form
//   R^0_{tuv} = sum_{a,b,c} C_t^a C_u^b C_v^c X^{t-2a} Y^{u-2b} Z^{v-2c} G_{t+u+v-a-b-c}
// (G_n = pref (-2 alpha)^n F_n; same values as eq. R_recursion) and used at
// once for every (P, Q) with P + Q = N:  Jh_P += R_N Dt_Q   (eq. j_formula).
#pragma once
#include "kern_args.hpp"
#include "md_device.hpp"

namespace md {

__host__ __device__ constexpr double hcoef(int t, int a)
{
    // t! / (a! (t-2a)! 2^a)
    double v = 1.0;
    for (int k = 0; k < a; ++k) v = v * (double)((t - 2 * k) * (t - 2 * k - 1)) / (2.0 * (k + 1));
    return v;
}

template <int LX, int LY>
__device__ __forceinline__ void jeng_quartet_stream(const double *G, const double *px, const double *py,
                                                    const double *pz, const double *dq, double *Jh)
{
    constexpr int L = LX + LY;
    static_for<0, nherm(L)>([&](auto Nc) {
        constexpr int N = decltype(Nc)::value;
        constexpr int t = herm_t(N), u = herm_u(N), v = herm_v(N);
        double r = 0.0;
        static_for<0, t / 2 + 1>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            static_for<0, u / 2 + 1>([&](auto bc) {
                constexpr int b = decltype(bc)::value;
                double rz = 0.0;
                static_for<0, v / 2 + 1>([&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    rz += hcoef(v, c) * pz[v - 2 * c] * G[t + u + v - a - b - c];
                });
                r += hcoef(t, a) * hcoef(u, b) * px[t - 2 * a] * py[u - 2 * b] * rz;
            });
        });
        // scatter: P + Q = N, P in H(LX), Q in H(LY)
        static_for<0, t + 1>([&](auto pxc) {
            constexpr int p1 = decltype(pxc)::value;
            static_for<0, u + 1>([&](auto pyc) {
                constexpr int p2 = decltype(pyc)::value;
                static_for<0, v + 1>([&](auto pzc) {
                    constexpr int p3 = decltype(pzc)::value;
                    if constexpr (p1 + p2 + p3 <= LX && (t - p1) + (u - p2) + (v - p3) <= LY) {
                        Jh[herm_idx(p1, p2, p3)] += r * dq[herm_idx(t - p1, u - p2, v - p3)];
                    }
                });
            });
        });
    });
}

}  // namespace md
