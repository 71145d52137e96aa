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

template <int LX, int LY>
__global__ __launch_bounds__(64) void jeng_reg(JArgs a)
{
    constexpr int L = LX + LY, NX = nherm(LX), NY = nherm(LY);
    const int g = blockIdx.x * 64 + threadIdx.x;
    const bool valid = g < a.nbp;
    const int gi = valid ? g : a.nbp - 1;
    const PrimPair pb = a.pp[a.pbase + gi];
    const double Qi = valid ? a.Qbra[a.owner[gi]] : 0.0;
    const double qi = valid ? pb.q : 0.0;
    int lo = 0, hi = a.nket;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (Qi * a.Qket[mid] >= a.tau) lo = mid + 1; else hi = mid;
    }
    const int nv = valid ? lo : 0;
    int nvmax = nv;
    double qmax = qi;
    for (int off = 32; off > 0; off >>= 1) {
        nvmax = max(nvmax, __shfl_xor(nvmax, off));
        qmax = fmax(qmax, __shfl_xor(qmax, off));
    }
    nvmax = __builtin_amdgcn_readfirstlane(nvmax);
    {
        const uint64_t bq = __double_as_longlong(qmax);
        const uint32_t lo32 = __builtin_amdgcn_readfirstlane((uint32_t)bq);
        const uint32_t hi32 = __builtin_amdgcn_readfirstlane((uint32_t)(bq >> 32));
        qmax = __longlong_as_double(((uint64_t)hi32 << 32) | lo32);
    }
    const int j0 = blockIdx.y * a.kchunk;
    const int j1 = min(min(a.nket, j0 + a.kchunk), nvmax);

    double Jh[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) Jh[i] = 0.0;
    for (int j = j0; j < j1; ++j) {
        const CPair B = a.ket[j];
        for (int kp = 0; kp < B.np; ++kp) {
            const PrimPair pk = a.pp[B.poff + kp];
            if (qmax * pk.q < a.tau_prim) break;
            if (j < nv && qi * pk.q >= a.tau_prim) {
                const double p = pb.p, q = pk.p, rpq = 1.0 / (p + q), alpha = p * q * rpq;
                const double X = pb.P[0] - pk.P[0], Y = pb.P[1] - pk.P[1], Z = pb.P[2] - pk.P[2];
                double F[L + 1];
                boys_all<L>(alpha * (X * X + Y * Y + Z * Z), F, a.boys);
                double G[L + 1], px[L + 1], py[L + 1], pz[L + 1];
                double s = kTwoPi52 * pb.K * pk.K / (p * q) * sqrt(rpq);
                const double m2a = -2.0 * alpha;
                px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
                for (int m = 0; m <= L; ++m) {
                    G[m] = s * F[m];
                    s *= m2a;
                }
#pragma unroll
                for (int m = 1; m <= L; ++m) {
                    px[m] = px[m - 1] * X;
                    py[m] = py[m - 1] * Y;
                    pz[m] = pz[m - 1] * Z;
                }
                const double *__restrict__ dt = a.Dt + (int64_t)(B.poff + kp - a.dt_base) * NY;
                double dq[NY];
#pragma unroll
                for (int k = 0; k < NY; ++k) dq[k] = dt[k];
                jeng_quartet_stream<LX, LY>(G, px, py, pz, dq, Jh);
            }
        }
    }
    if (valid && j1 > j0) {
#pragma unroll
        for (int P = 0; P < NX; ++P) unsafeAtomicAdd(&a.Jh[(int64_t)g * NX + P], Jh[P]);
    }
}

// register J-engine is used where its live set (Hermite J, Hermite density,
// Boys values and coordinate powers) stays within about 115 doubles
__host__ __device__ constexpr bool jeng_reg_ok(int lx, int ly)
{
    return lx + ly >= 6 && nherm(lx) + nherm(ly) + 4 * (lx + ly + 1) <= 116;
}

template <int LX, int LY>
void jeng_reg_launch_t(const JArgs &a, hipStream_t st)
{
    const int nch = (a.nket + a.kchunk - 1) / a.kchunk;
    if (a.nbp <= 0 || nch <= 0) return;
    dim3 grid((a.nbp + 63) / 64, nch);
    hipLaunchKernelGGL((jeng_reg<LX, LY>), grid, dim3(64), 0, st, a);
}

}  // namespace md
