// wave_r.hpp -- one 64-lane wavefront (one workgroup) builds the auxiliary
// integrals R^0_{tuv} of a single primitive quartet in LDS (eq. R_recursion):
// lane m <= L evaluates F_m, then the recursion runs level by level
// (R^{n}_{...} from R^{n+1}_{...}) with the entries of a level spread over the
// lanes.  Level 0 is written densely, sR0[(t*(L+1)+u)*(L+1)+v], so that the
// address of R_{P+Q} is the sum of the addresses of P and Q.
#pragma once
#include "md_common.hpp"
#include "md_device.hpp"

namespace md {

// packed (t | u<<8 | v<<16) of shell-ordered Hermite indices, n <= 14
struct HermDecode {
    int32_t tuv[nherm(14)];
    constexpr HermDecode() : tuv()
    {
        for (int k = 0; k < nherm(14); ++k) tuv[k] = herm_t(k) | (herm_u(k) << 8) | (herm_v(k) << 16);
    }
};
__constant__ const HermDecode c_herm{};

__device__ __forceinline__ int herm_idx_rt(int t, int u, int v)
{
    int n = t + u + v, s = u + v;
    return n * (n + 1) * (n + 2) / 6 + s * (s + 1) / 2 + v;
}

// Geometry of one primitive quartet; the same on every lane.
// c, w, pref0 and r serve the scaled single-precision form (md_device.hpp):
// c = sqrt(2p), w = -q/(p+q), pref0 = 2 pi^{5/2}/(pq sqrt(p+q)), r = sqrt(p/q).
// With the long-range operator erf(omega r)/r (om2 = omega^2 > 0), alpha, T
// and w carry the factor s0 = omega^2/(alpha + omega^2) and the prefactors
// sqrt(s0) (eq. eri_longrange_formula).
struct QuartetGeo {
    double X, Y, Z, T, alpha, pref;
    double c, w, pref0, r;
};

__device__ __forceinline__ QuartetGeo quartet_geo(const PrimPair &pb, const PrimPair &pk, double om2)
{
    QuartetGeo g;
    double p = pb.p, q = pk.p;
    const double rs = rsqrt(p + q);  // 1/(pq) from the stored 1/(2p), 1/(2q)
    double rpq = rs * rs;
    g.alpha = p * q * rpq;
    g.X = pb.P[0] - pk.P[0];
    g.Y = pb.P[1] - pk.P[1];
    g.Z = pb.P[2] - pk.P[2];
    g.T = g.alpha * (g.X * g.X + g.Y * g.Y + g.Z * g.Z);
    g.pref0 = kTwoPi52 * (4.0 * pb.o2p * pk.o2p) * rs;
    g.w = -q * rpq;
    if (om2 > 0.0) {  // long-range operator (eq. eri_longrange_formula)
        const double s0 = om2 / (g.alpha + om2);
        g.alpha *= s0;
        g.T *= s0;
        g.w *= s0;
        g.pref0 *= sqrt(s0);
    }
    g.pref = g.pref0 * pb.K * pk.K;
    g.c = sqrt(2.0 * p);
    g.r = sqrt(p / q);
    return g;
}

// The fields of a ket primitive pair that a quartet needs, loaded one by one
// (a loop-carried copy of the whole record would live in scratch memory).
struct PairLite {
    double p, K, q, P0, P1, P2, o2p;
};

__device__ __forceinline__ PairLite pair_lite(const PrimPair *__restrict__ r)
{
    PairLite x;
    x.p = r->p;
    x.o2p = r->o2p;
    x.K = r->K;
    x.q = r->q;
    x.P0 = r->P[0];
    x.P1 = r->P[1];
    x.P2 = r->P[2];
    return x;
}

__device__ __forceinline__ QuartetGeo quartet_geo(const PrimPair &pb, const PairLite &pk, double om2)
{
    QuartetGeo g;
    double p = pb.p, q = pk.p;
    const double rs = rsqrt(p + q);
    double rpq = rs * rs;
    g.alpha = p * q * rpq;
    g.X = pb.P[0] - pk.P0;
    g.Y = pb.P[1] - pk.P1;
    g.Z = pb.P[2] - pk.P2;
    g.T = g.alpha * (g.X * g.X + g.Y * g.Y + g.Z * g.Z);
    g.pref0 = kTwoPi52 * (4.0 * pb.o2p * pk.o2p) * rs;
    g.w = -q * rpq;
    if (om2 > 0.0) {  // long-range operator (eq. eri_longrange_formula)
        const double s0 = om2 / (g.alpha + om2);
        g.alpha *= s0;
        g.T *= s0;
        g.w *= s0;
        g.pref0 *= sqrt(s0);
    }
    g.pref = g.pref0 * pb.K * pk.K;
    g.c = sqrt(2.0 * p);
    g.r = sqrt(p / q);
    return g;
}

// Phase 1 (no barrier inside): lane m <= L writes sF[m] = pref (-2 alpha)^m F_m
// (single precision: the scaled G~_m = pref0 w^m F_m).  F_m and the scale are
// formed in double precision; the product is stored as T.
// x^n for 0 <= n <= NMAX by binary powering: the same steps for every lane
// (a loop of n multiplications runs to the wavefront's largest n).
template <int NMAX, typename V>
__device__ __forceinline__ V pow_small(V x, int n)
{
    V v = V(1);
#pragma unroll
    for (int bit = 1; bit <= NMAX; bit <<= 1) {
        if (n & bit) v *= x;
        x *= x;
    }
    return v;
}

template <int L, typename T>
__device__ __forceinline__ void wave_boys(const QuartetGeo &g, const double *__restrict__ btab,
                                          T *sF, int lane)
{
    if (lane <= L) {
        double F = boys_one(lane, g.T, btab);
        const double s = sizeof(T) == 4 ? g.pref0 : g.pref, m2a = sizeof(T) == 4 ? g.w : -2.0 * g.alpha;
        sF[lane] = (T)(s * pow_small<L>(m2a, lane) * F);
    }
}

// Phase 2: recursion; sF must be visible (barrier before the call).  Ends
// with a barrier; afterwards sR0 holds the dense level-0 table.
template <int L>
__device__ __forceinline__ void wave_recur(const QuartetGeo &g, const double *sF, double *sLa,
                                           double *sLb, double *sR0, int lane)
{
    constexpr int L1 = L + 1;
    if constexpr (L == 0) {
        if (lane == 0) sR0[0] = sF[0];
        __syncthreads();
        return;
    } else {
        const double *prev = sF + L;  // level L holds only (0,0,0)
        int which = 0;
        for (int n = L - 1; n >= 0; --n) {
            const int cnt = nherm(L - n);
            double *out = which ? sLb : sLa;
            for (int k = lane; k < cnt; k += 64) {
                const int code = c_herm.tuv[k];
                const int t = code & 0xff, u = (code >> 8) & 0xff, v = code >> 16;
                double val;
                if (k == 0) {
                    val = sF[n];
                } else if (t > 0) {
                    val = g.X * prev[herm_idx_rt(t - 1, u, v)];
                    if (t > 1) val += (double)(t - 1) * prev[herm_idx_rt(t - 2, u, v)];
                } else if (u > 0) {
                    val = g.Y * prev[herm_idx_rt(t, u - 1, v)];
                    if (u > 1) val += (double)(u - 1) * prev[herm_idx_rt(t, u - 2, v)];
                } else {
                    val = g.Z * prev[herm_idx_rt(t, u, v - 1)];
                    if (v > 1) val += (double)(v - 1) * prev[herm_idx_rt(t, u, v - 2)];
                }
                if (n == 0)
                    sR0[(t * L1 + u) * L1 + v] = val;
                else
                    out[k] = val;
            }
            __syncthreads();
            prev = out;
            which ^= 1;
        }
    }
}

// 1D Hermite coefficient table of one axis into LDS, layout [i][j][t] with
// dims (LA+1, LB+1, LA+LB+1); E^{00}_0 = 1 (eq. E_recursion).
template <int LA, int LB>
__device__ __forceinline__ void etab_lds(double PA, double PB, double o2p, double *E)
{
    constexpr int DJ = LA + LB + 1, DI = (LB + 1) * DJ;
    for (int i = 0; i <= LA; ++i)
        for (int j = 0; j <= LB; ++j)
            for (int t = 0; t < DJ; ++t) E[i * DI + j * DJ + t] = 0.0;
    E[0] = 1.0;
    for (int i = 0; i < LA; ++i)
        for (int t = 0; t <= i + 1; ++t) {
            double v = (t <= i) ? PA * E[i * DI + t] : 0.0;
            if (t > 0) v += o2p * E[i * DI + t - 1];
            if (t + 1 <= i) v += (double)(t + 1) * E[i * DI + t + 1];
            E[(i + 1) * DI + t] = v;
        }
    for (int i = 0; i <= LA; ++i)
        for (int j = 0; j < LB; ++j)
            for (int t = 0; t <= i + j + 1; ++t) {
                double v = (t <= i + j) ? PB * E[i * DI + j * DJ + t] : 0.0;
                if (t > 0) v += o2p * E[i * DI + j * DJ + t - 1];
                if (t + 1 <= i + j) v += (double)(t + 1) * E[i * DI + j * DJ + t + 1];
                E[i * DI + (j + 1) * DJ + t] = v;
            }
}


// Closed form of the recursion (same values as eq. R_recursion): with
// G_n = pref (-2 alpha)^n F_n and s = X^2+Y^2+Z^2, dG_n/ds = G_{n+1}/2, so
//   R^0_{tuv} = sum_{a<=t/2, b<=u/2, c<=v/2} C_t^a C_u^b C_v^c
//               X^{t-2a} Y^{u-2b} Z^{v-2c} G_{t+u+v-a-b-c},
//   C_t^a = t! / (a! (t-2a)! 2^a).
// Every entry is independent, so the lanes of a wave fill the table with one
// barrier instead of one per recursion level.
template <typename T>
struct HermCoef {
    T c[15][8];
    constexpr HermCoef() : c()
    {
        for (int t = 0; t < 15; ++t) {
            double v = 1.0;  // a = 0
            for (int a = 0; 2 * a <= t && a < 8; ++a) {
                c[t][a] = (T)v;
                v = v * (double)((t - 2 * a) * (t - 2 * a - 1)) / (2.0 * (a + 1));
            }
        }
    }
};
__constant__ const HermCoef<double> c_hcoef{};
__constant__ const HermCoef<float> c_hcoef_f{};
template <typename T>
__device__ __forceinline__ const HermCoef<T> &hcoef_table()
{
    if constexpr (sizeof(T) == 4) return c_hcoef_f; else return c_hcoef;
}

// Phase 1 helper: lane 0..L also stores the powers X^k, Y^k, Z^k into sPow
// (layout [axis][L+1]); call together with wave_boys (before the barrier).
// (single precision: powers of the scaled c X, c Y, c Z)
template <int L, typename T>
__device__ __forceinline__ void wave_powers(const QuartetGeo &g, T *sPow, int lane)
{
    if (lane <= L) {
        double px = 1.0, py = 1.0, pz = 1.0;
        const double f = sizeof(T) == 4 ? g.c : 1.0;
        const double X = f * g.X, Y = f * g.Y, Z = f * g.Z;
        for (int k = 0; k < lane; ++k) {
            px *= X;
            py *= Y;
            pz *= Z;
        }
        sPow[lane] = (T)px;
        sPow[(L + 1) + lane] = (T)py;
        sPow[2 * (L + 1) + lane] = (T)pz;
    }
}

// Phase 2 (after the barrier that publishes sF and sPow): dense R^0 into sR0.
// No barrier inside.
template <int L, typename T>
__device__ __forceinline__ void wave_r0(const T *sF, const T *sPow, T *sR0, int lane)
{
    constexpr int L1 = L + 1;
    const HermCoef<T> &hc = hcoef_table<T>();
    for (int k = lane; k < nherm(L); k += 64) {
        const int code = c_herm.tuv[k];
        const int t = code & 0xff, u = (code >> 8) & 0xff, v = code >> 16;
        T acc = T(0);
        for (int a = 0; 2 * a <= t; ++a) {
            const T ca = hc.c[t][a] * sPow[t - 2 * a];
            for (int b = 0; 2 * b <= u; ++b) {
                const T cab = ca * hc.c[u][b] * sPow[L1 + u - 2 * b];
                const int n0 = t + u + v - a - b;
                for (int c = 0; 2 * c <= v; ++c)
                    acc += cab * hc.c[v][c] * sPow[2 * L1 + v - 2 * c] * sF[n0 - c];
            }
        }
        sR0[(t * L1 + u) * L1 + v] = acc;
    }
}

// One axis of the 1D Hermite tables computed in registers (eq. E_recursion)
// and stored to LDS with the [i][j][t] layout of etab_lds.
template <int LA, int LB>
__device__ __forceinline__ void etab_reg_store(double PA, double PB, double o2p, double *E)
{
    constexpr int DJ = LA + LB + 1, DI = (LB + 1) * DJ;
    Etab<LA, LB> T;
    etab_build<LA, LB>(PA, PB, o2p, T);
    static_for<0, LA + 1>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        static_for<0, LB + 1>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            static_for<0, DJ>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                E[i * DI + j * DJ + t] = (t <= i + j) ? T.e[i][j][t] : 0.0;
            });
        });
    });
}

// LDS-resident form of the closed form above, for the wave kernels.
// Per quartet, lanes tabulate the per-axis factors
//     sH[axis][t][a] = C_t^a X_axis^{t-2a},   t <= L, a <= t/2
// (single precision: the scaled X~ = c X) in the same phase as the Boys
// values, so that building R reads LDS only:
//     R^0_{tuv} = sum_{a,b,c} sH[x][t][a] sH[y][u][b] sH[z][v][c] G_{t+u+v-a-b-c}.
template <int L>
struct HPolyDims {
    static constexpr int H = L / 2 + 1;
    static constexpr int N = 3 * (L + 1) * H;
};

// Hermite index decode table (t | u<<8 | v<<16 for k < n) into LDS; call once
// at kernel start, visible after the first barrier.
__device__ __forceinline__ void herm_table_lds(int *sHerm, int n, int lane)
{
    for (int k = lane; k < n; k += 64) sHerm[k] = c_herm.tuv[k];
}

// Phase 1 (no barrier inside).
template <int L, typename T>
__device__ __forceinline__ void wave_hpoly(const QuartetGeo &g, T *sH, int lane)
{
    constexpr int H = HPolyDims<L>::H;
    const double f = sizeof(T) == 4 ? g.c : 1.0;
    const double gx = f * g.X, gy = f * g.Y, gz = f * g.Z;  // values, not a runtime-indexed member
    for (int i = lane; i < HPolyDims<L>::N; i += 64) {
        const int axis = i / ((L + 1) * H), t = (i / H) % (L + 1), a = i % H;
        if (2 * a > t) {  // no such term: a zero the planned R^0 sums can point at
            sH[i] = T(0);
            continue;
        }
        double x = gx;
        if (axis == 1) x = gy;
        if (axis == 2) x = gz;
        // c x^m, m = t - 2a <= L, by binary powering over the bits of m (the
        // same steps for every lane instead of a loop of m multiplications)
        const int m = t - 2 * a;
        double v = c_hcoef.c[t][a];
#pragma unroll
        for (int bit = 1; bit <= L; bit <<= 1) {
            if (m & bit) v *= x;
            x *= x;
        }
        sH[i] = (T)v;
    }
}

// largest number of closed-form terms (a, b, c) over the Hermite indices
// k in [k0, k1): (t/2 + 1)(u/2 + 1)(v/2 + 1)
__host__ __device__ constexpr int r0_terms_max(int k0, int k1)
{
    int m = 0;
    for (int k = k0; k < k1; ++k) {
        const int v = (herm_t(k) / 2 + 1) * (herm_u(k) / 2 + 1) * (herm_v(k) / 2 + 1);
        if (v > m) m = v;
    }
    return m;
}

// Hermite indices of R^0 of order L in the order the wavefront builds them:
// by number of closed-form terms, largest first, so that each round of 64
// lanes holds entries of similar term counts and the flat walk's trip count
// (the round's largest) wastes few slots; tm[r] is that count for round r,
// off[r] the first term slot of round r in a plan.
template <int L>
struct R0Rounds {
    static constexpr int NH = nherm(L), NR = (NH + 63) / 64;
    int perm[NH], tm[NR], off[NR + 1], tmax;
    constexpr R0Rounds() : perm(), tm(), off(), tmax(0)
    {
        int n[NH] = {}, nmax = 0;
        for (int k = 0; k < NH; ++k) {
            n[k] = (herm_t(k) / 2 + 1) * (herm_u(k) / 2 + 1) * (herm_v(k) / 2 + 1);
            if (n[k] > nmax) nmax = n[k];
        }
        int i = 0;  // stable, by descending term count
        for (int c = nmax; c >= 1; --c)
            for (int k = 0; k < NH; ++k)
                if (n[k] == c) perm[i++] = k;
        off[0] = 0;
        for (int r = 0; r < NR; ++r) {
            tm[r] = 0;
            for (int q = r * 64; q < NH && q < r * 64 + 64; ++q)
                if (n[perm[q]] > tm[r]) tm[r] = n[perm[q]];
            off[r + 1] = off[r] + tm[r];
            if (tm[r] > tmax) tmax = tm[r];
        }
    }
};

// Hermite index of lane slot q = 64 r + lane in build order (constant table).
template <int L>
__device__ __forceinline__ int r0_perm(int q)
{
    static constexpr R0Rounds<L> RR{};
    return RR.perm[q];
}

// Phase 2 (after the barrier that publishes sF, sH and sHerm): dense R^0
// into sR0 at t ST + u SU + v (by default the cube (L+1)^3).  No barrier inside.  Each lane walks the (a, b, c) terms of its
// entry in one flat loop whose trip count is the round's largest term
// count, the same for every lane (nested per-lane loops would run the union
// of all lanes' term boxes).
template <int L, typename T, int ST = (L + 1) * (L + 1), int SU = L + 1>
__device__ __forceinline__ void wave_r0h(const T *sF, const T *sH, const int *sHerm, T *sR0, int lane)
{
    constexpr int L1 = L + 1, H = HPolyDims<L>::H, NH = nherm(L);
    const T *hx = sH, *hy = sH + L1 * H, *hz = sH + 2 * L1 * H;
    static_for<0, (NH + 63) / 64>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        constexpr int TM = R0Rounds<L>().tm[r];
        const int q = r * 64 + lane;
        if (q < NH) {
            const int code = sHerm[r0_perm<L>(q)];
            const int t = code & 0xff, u = (code >> 8) & 0xff, v = code >> 16;
            const int nb = u / 2 + 1, nc = v / 2 + 1, nterm = (t / 2 + 1) * nb * nc;
            const T *px = hx + t * H, *py = hy + u * H, *pz = hz + v * H;
            const T *pf = sF + t + u + v;
            T acc = T(0);
            int a = 0, b = 0, c = 0;
#pragma unroll 2
            for (int st = 0; st < TM; ++st) {
                if (st < nterm) acc += px[a] * py[b] * pz[c] * pf[-(a + b + c)];
                if (++c == nc) {
                    c = 0;
                    if (++b == nb) {
                        b = 0;
                        ++a;
                    }
                }
            }
            sR0[t * ST + u * SU + v] = acc;
        }
    });
}

// The same closed form with the term walk planned once per kernel: for the
// entry of lane slot 64 r + lane (build order, R0Rounds) and each of the
// round's term slots j, one word in LDS (code[(off_r + j) 64 + lane]) packs
// the offsets of the term's x, y and z Hermite-polynomial entries and of its
// G value, 8 bits each (slots past the entry's term count point at a zero
// polynomial entry), so that each term costs five LDS reads, the field
// extractions and three multiply-adds instead of the flat loop's index
// bookkeeping.  The offsets are in bytes while one axis row of sH takes at
// most 256 bytes, else in elements; used for L <= 9 (the plan takes 5 KB of
// LDS or less).  Same terms in the same order as wave_r0h, so the same sums.
template <int L, typename T>
struct R0Plan {
    static constexpr int H = HPolyDims<L>::H, NH = nherm(L), NR = (NH + 63) / 64;
    static constexpr bool OK = L >= 2 && L <= 9;
    static constexpr bool BYTES = (L + 1) * H * (int)sizeof(T) <= 256;  // offsets in bytes, else in elements
    static constexpr int NT = R0Rounds<L>().off[NR], TMAX = R0Rounds<L>().tmax;
    uint32_t *code;  // LDS, NT x 64 words
    int out[NR];     // R^0 index t ST + u SU + v of the lane's entry, -1 if none
};

template <int L, typename T, int ST = (L + 1) * (L + 1), int SU = L + 1>
__device__ __forceinline__ void r0_plan_build(R0Plan<L, T> &p, int lane)
{
    using P = R0Plan<L, T>;
    constexpr R0Rounds<L> RR{};
    constexpr int H = P::H, B = P::BYTES ? (int)sizeof(T) : 1;
    constexpr uint32_t ZERO = (uint32_t)((H - 1) * B);  // x entry (t = 0, a = H - 1): zero
#pragma unroll
    for (int r = 0; r < P::NR; ++r) {
        const int q = r * 64 + lane;
        int t = 0, u = 0, v = 0;
        const bool ok = q < P::NH;
        if (ok) {
            const int code = c_herm.tuv[r0_perm<L>(q)];
            t = code & 0xff;
            u = (code >> 8) & 0xff;
            v = code >> 16;
        }
        p.out[r] = ok ? t * ST + u * SU + v : -1;
        const int nb = u / 2 + 1, nc = v / 2 + 1, nterm = ok ? (t / 2 + 1) * nb * nc : 0;
        int a = 0, b = 0, c = 0;
#pragma unroll
        for (int j = 0; j < P::TMAX; ++j) {
            if (j < RR.tm[r]) {
                uint32_t w = ZERO;
                if (j < nterm)
                    w = (uint32_t)((t * H + a) * B) | ((uint32_t)((u * H + b) * B) << 8) |
                        ((uint32_t)((v * H + c) * B) << 16) | ((uint32_t)((t + u + v - a - b - c) * B) << 24);
                p.code[(RR.off[r] + j) * 64 + lane] = w;
                if (++c == nc) {
                    c = 0;
                    if (++b == nb) {
                        b = 0;
                        ++a;
                    }
                }
            }
        }
    }
}

template <int L, typename T, int ST = (L + 1) * (L + 1), int SU = L + 1>
__device__ __forceinline__ void wave_r0h_plan(const R0Plan<L, T> &p, const T *sF, const T *sH, T *sR0, int lane)
{
    using P = R0Plan<L, T>;
    constexpr R0Rounds<L> RR{};
    constexpr int ROW = (L + 1) * P::H;
    const char *hx = (const char *)sH, *hy = (const char *)(sH + ROW), *hz = (const char *)(sH + 2 * ROW);
    const char *f = (const char *)sF;
    constexpr uint32_t M = P::BYTES ? 1u : (uint32_t)sizeof(T);
#pragma unroll
    for (int r = 0; r < P::NR; ++r) {
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < P::TMAX; ++j) {
            if (j < RR.tm[r]) {
                const uint32_t w = p.code[(RR.off[r] + j) * 64 + lane];
                const T x = *(const T *)(hx + (w & 0xffu) * M);
                const T y = *(const T *)(hy + ((w >> 8) & 0xffu) * M);
                const T z = *(const T *)(hz + ((w >> 16) & 0xffu) * M);
                const T g = *(const T *)(f + (w >> 24) * M);
                acc += x * y * z * g;
            }
        }
        if (p.out[r] >= 0) sR0[p.out[r]] = acc;
    }
}

// One axis of the 1D Hermite tables built in registers (eq. E_recursion, in
// double) and stored to LDS as T with the [i][j][t] layout of etab_lds minus
// the padding: dims (LA+1, LB+1, LA+LB+1), entries multiplied by k c^t.
template <int LA, int LB, typename T>
__device__ __forceinline__ void etab_store_scaled(double PA, double PB, double o2p, double k, double c, T *E)
{
    constexpr int DJ = LA + LB + 1, DI = (LB + 1) * DJ;
    Etab<LA, LB> Tb;
    etab_build<LA, LB>(PA, PB, o2p, Tb);
    double w[LA + LB + 1];
    w[0] = k;
    for (int t = 1; t <= LA + LB; ++t) w[t] = w[t - 1] * c;
    static_for<0, LA + 1>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        static_for<0, LB + 1>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            static_for<0, DJ>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                E[i * DI + j * DJ + t] = (T)((t <= i + j) ? Tb.e[i][j][t] * w[t] : 0.0);
            });
        });
    });
}

// Cartesian exponents of component c of a shell with angular momentum l (runtime).
__device__ __forceinline__ void cart_rt(int l, int c, int &x, int &y, int &z)
{
    // components ordered x descending: c = (l-x)(l-x+1)/2 + (l-x-y)
    int s = 0;
    while ((s + 1) * (s + 2) / 2 <= c) ++s;
    x = l - s;
    z = c - s * (s + 1) / 2;
    y = s - z;
}

}  // namespace md
