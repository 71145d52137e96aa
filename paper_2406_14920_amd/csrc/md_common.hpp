// md_common.hpp -- shared device/host definitions of the MI355X J/K library.
//
// Hermite index conventions follow the McMurchie-Davidson scheme of
// arXiv 2406.14920 (eqs. cartesian_to_hermite, E_recursion, R_recursion):
// a Hermite index (t,u,v) with t+u+v <= L is stored "by shells", n = t+u+v
// ascending, inside a shell t descending then u descending.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace md {

constexpr double kPi = 3.14159265358979323846264338327950288;

__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }
__host__ __device__ constexpr int nherm(int L) { return L < 0 ? 0 : (L + 1) * (L + 2) * (L + 3) / 6; }
__host__ __device__ constexpr int nsph(int l) { return 2 * l + 1; }
__host__ __device__ constexpr int herm_idx(int t, int u, int v)
{
    return nherm(t + u + v - 1) + (u + v) * (u + v + 1) / 2 + v;
}
// decode a shell-ordered Hermite index
__host__ __device__ constexpr int herm_n(int k)
{
    int n = 0;
    while (nherm(n) <= k) ++n;
    return n;
}
__host__ __device__ constexpr int herm_t(int k)
{
    int n = herm_n(k), r = k - nherm(n - 1);
    int s = 0;  // s = u+v
    while ((s + 1) * (s + 2) / 2 <= r) ++s;
    return n - s;
}
__host__ __device__ constexpr int herm_v(int k)
{
    int n = herm_n(k), r = k - nherm(n - 1);
    int s = 0;
    while ((s + 1) * (s + 2) / 2 <= r) ++s;
    return r - s * (s + 1) / 2;
}
__host__ __device__ constexpr int herm_u(int k) { return herm_n(k) - herm_t(k) - herm_v(k); }

// Cartesian components of a shell, lexicographic with x power descending
__host__ __device__ constexpr int cart_x(int l, int c)
{
    int n = 0;
    for (int i = l; i >= 0; --i)
        for (int j = l - i; j >= 0; --j) {
            if (n == c) return i;
            ++n;
        }
    return 0;
}
__host__ __device__ constexpr int cart_y(int l, int c)
{
    int n = 0;
    for (int i = l; i >= 0; --i)
        for (int j = l - i; j >= 0; --j) {
            if (n == c) return j;
            ++n;
        }
    return 0;
}
__host__ __device__ constexpr int cart_z(int l, int c) { return l - cart_x(l, c) - cart_y(l, c); }

// number of non-zero Hermite terms of one Cartesian pair component
__host__ __device__ constexpr int box_nnz(int la, int ca, int lb, int cb)
{
    return (cart_x(la, ca) + cart_x(lb, cb) + 1) * (cart_y(la, ca) + cart_y(lb, cb) + 1) *
           (cart_z(la, ca) + cart_z(lb, cb) + 1);
}

// largest box over the pair components ab in [ab0, ab1) (components ab = i NB + j)
__host__ __device__ constexpr int box_max(int la, int lb, int ab0, int ab1)
{
    const int nb = ncart(lb), nab = ncart(la) * nb;
    int m = 0;
    for (int ab = ab0; ab < ab1 && ab < nab; ++ab) {
        const int v = box_nnz(la, ab / nb, lb, ab % nb);
        if (v > m) m = v;
    }
    return m;
}

// ---------------------------------------------------------------------------
// Pair records (HBM, array-of-structures, 128 B per primitive pair)
// ---------------------------------------------------------------------------
struct alignas(16) PrimPair {
    double a, b;     // exponents of the first / second shell
    double p;        // a + b
    double K;        // C_a C_b exp(-ab/p |A-B|^2): coefficients and Gaussian product prefactor
    double P[3];     // pair centre (eq. pair_definition)
    double PA[3];    // P - A
    double PB[3];    // P - B
    double q;        // primitive Schwarz bound sqrt(max |(ij|ij)|)
    double o2p;      // 1 / (2p)
    double pad;
};
static_assert(sizeof(PrimPair) == 128, "PrimPair must be 128 bytes");

struct alignas(16) CPair {
    int32_t sh1, sh2;   // shells, l(sh1) >= l(sh2)
    int32_t poff, np;   // first primitive pair, number of primitive pairs
    int32_t c1, c2;     // Cartesian AO offsets of sh1 / sh2
    int32_t at1, at2;   // atoms of sh1 / sh2
};
static_assert(sizeof(CPair) == 32, "CPair must be 32 bytes");

// ---------------------------------------------------------------------------
// Boys function table: F_m(T_i) on T_i = i*h, i = 0..kBoysNG-1, m = 0..kBoysNM-1,
// row-major [i][m] with row stride kBoysNC; column kBoysNM of a row holds
// e^{-T_i}.  Taylor expansion around the nearest grid point (dF_m/dT =
// -F_{m+1}) with kBoysK terms, then downward recursion with
// e^{-T} = e^{-T_i} e^{T_i - T} (the last factor a Taylor polynomial, the step
// being at most h/2); beyond kBoysTmax the asymptotic F_0 = sqrt(pi/T)/2 and
// upward recursion.
// ---------------------------------------------------------------------------
constexpr double kBoysH = 0.1;
constexpr double kBoysTmax = 40.0;
constexpr int kBoysNG = 402;
constexpr int kBoysK = 8;
constexpr int kBoysNM = 24;  // orders available in the table (m + kBoysK - 1 < kBoysNM)
constexpr int kBoysNC = kBoysNM + 1;  // row stride: the orders, then e^{-T_i}

// e^x for |x| <= h/2 = 0.05: degree-8 Taylor polynomial, relative error
// below 0.05^9/9! ~ 5e-18
__device__ __forceinline__ double exp_small(double x)
{
    double s = 1.0 / 40320.0;
    s = 1.0 / 5040.0 + x * s;
    s = 1.0 / 720.0 + x * s;
    s = 1.0 / 120.0 + x * s;
    s = 1.0 / 24.0 + x * s;
    s = 1.0 / 6.0 + x * s;
    s = 0.5 + x * s;
    s = 1.0 + x * s;
    return 1.0 + x * s;
}

// All orders 0..M for a compile-time M.
template <int M>
__device__ __forceinline__ void boys_all(double T, double *F, const double *__restrict__ tab)
{
    if (T < kBoysTmax) {
        int i = (int)(T * (1.0 / kBoysH) + 0.5);
        double x = (double)i * kBoysH - T;  // step from the grid point, |x| <= h/2
        const double *row = tab + i * kBoysNC + M;
        double s = row[kBoysK - 1];
#pragma unroll
        for (int k = kBoysK - 2; k >= 0; --k) s = row[k] + s * x * (1.0 / (k + 1));
        F[M] = s;
        if (M > 0) {
            const double e = tab[i * kBoysNC + kBoysNM] * exp_small(x);
            double T2 = 2.0 * T;
#pragma unroll
            for (int m = M - 1; m >= 0; --m) F[m] = (T2 * F[m + 1] + e) * (1.0 / (2 * m + 1));
        }
    } else {
        double rT = 1.0 / T;
        F[0] = sqrt(0.25 * kPi * rT);
        if (M > 0) {
            double e = exp(-T);
            double h = 0.5 * rT;
#pragma unroll
            for (int m = 0; m < M; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) * h;
        }
    }
}

// A single order m (runtime) -- used when lanes evaluate different orders.
__device__ __forceinline__ double boys_one(int m, double T, const double *__restrict__ tab)
{
    if (T < kBoysTmax) {
        int i = (int)(T * (1.0 / kBoysH) + 0.5);
        double x = (double)i * kBoysH - T;
        const double *row = tab + i * kBoysNC + m;
        double s = row[kBoysK - 1];
#pragma unroll
        for (int k = kBoysK - 2; k >= 0; --k) s = row[k] + s * x * (1.0 / (k + 1));
        return s;
    }
    double rT = 1.0 / T;
    double F = sqrt(0.25 * kPi * rT);
    double e = exp(-T);
    double h = 0.5 * rT;
    for (int k = 0; k < m; ++k) F = ((2 * k + 1) * F - e) * h;
    return F;
}

// 2 pi^{5/2}
constexpr double kTwoPi52 = 34.98683665524972497;

}  // namespace md
