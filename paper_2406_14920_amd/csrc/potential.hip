// potential.hip -- one-electron integrals: overlap S, kinetic energy T and the
// point-charge potential V_mn = sum_C q_C int m(r) n(r) / |r - C|
// (nuclear attraction with q_C = -Z_C, or any point charges such as QM/MM
// embedding charges; eqs. v1e_definition, v1e_summation_over_C) and the
// derivatives of E_V = sum_mn P_mn V_mn (SI eqs. si_v1e_derivative_A/B/C).
//
// By eq. v1e_formula a primitive pair's Hermite potential is
//     Vh_t = K_ab (2 pi/p) sum_C q_C R^0_t(p, P - C),     t in H(L),
// with R from (-2p)^m F_m(p |P - C|^2) (eq. R_recursion).  One lane owns one
// primitive pair and walks a range of the charges (wave-uniform, so their
// coordinates arrive through scalar loads); the charges are split over
// blockIdx.y so that a class with few pairs still fills the chip, each split
// storing its sums for a fixed-order reduction.  The Cartesian pair block is
// then the J-engine's Hermite-to-Cartesian step.  With L = la + lb + 1 the
// same Hermite potential feeds the pair derivative of the Coulomb gradient
// kernel (d/dA, d/dB of every pair).  The derivative with respect to a charge
// position is (SI eq. si_v1e_derivative_C)
//     dE_V/dC_k = -sum_pairs K_ab (2 pi/p) q_C sum_t Dh_t R^0_{t+1_k}(p, P - C),
// Dh_t = f sum_ab P_ab E^{ab}_t the pair's Hermite density; there one lane
// owns one charge and walks a range of the pairs (wave-uniform), the pair
// ranges split over blockIdx.y with per-split partials reduced in order.
#include <algorithm>

#include "kern_args.hpp"
#include "launch.hpp"
#include "md_device.hpp"
#include "wave_r.hpp"

namespace md {

// Overlap and kinetic energy of one contracted pair, thread per Cartesian
// component (eqs. overlap_formula, kinetic_formula): with the one-direction
// Hermite coefficients E (E^{00}_0 = 1; K_ab kept apart) per primitive pair
//     S_ab += K_ab (pi/p)^{3/2} E^x_0 E^y_0 E^z_0,
//     T_ab += K_ab (pi/p)^{3/2} sum_k t_k prod_{other} E_0,
//     t_k = (2j+1) b E^{i,j}_0 - 2 b^2 E^{i,j+2}_0 - j(j-1)/2 E^{i,j-2}_0,
// written as one triangle of the accumulators (X = Acc + Acc^T).
template <int LA, int LB>
__global__ __launch_bounds__(128) void st_pair(const CPair *__restrict__ cp, int ncp,
                                               const PrimPair *__restrict__ pp, double *__restrict__ Sacc,
                                               double *__restrict__ Tacc, int ld)
{
    constexpr int NA = ncart(LA), NB = ncart(LB), LB2 = LB + 2;
    constexpr int DJ = LA + LB2 + 1, DI = (LB2 + 1) * DJ, EBD = (LA + 1) * DI;
    __shared__ double sE[3 * EBD];
    const int c = blockIdx.x;
    if (c >= ncp) return;
    const CPair A = cp[c];
    const int tid = threadIdx.x;
    int ia[3] = {0, 0, 0}, jb[3] = {0, 0, 0};
    if (tid < NA * NB) {
        cart_rt(LA, tid / NB, ia[0], ia[1], ia[2]);
        cart_rt(LB, tid % NB, jb[0], jb[1], jb[2]);
    }
    double sacc = 0.0, tacc = 0.0;
    for (int ip = 0; ip < A.np; ++ip) {
        const PrimPair pb = pp[A.poff + ip];
        if (tid < 3) {
            const double pa = tid == 0 ? pb.PA[0] : (tid == 1 ? pb.PA[1] : pb.PA[2]);
            const double pbb = tid == 0 ? pb.PB[0] : (tid == 1 ? pb.PB[1] : pb.PB[2]);
            etab_lds<LA, LB2>(pa, pbb, pb.o2p, sE + tid * EBD);
        }
        __syncthreads();
        if (tid < NA * NB) {
            const double b = pb.b;
            double sk[3], tk[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double *E = sE + k * EBD + ia[k] * DI;
                const int j = jb[k];
                sk[k] = E[j * DJ];
                double t = (2 * j + 1) * b * E[j * DJ] - 2.0 * b * b * E[(j + 2) * DJ];
                if (j >= 2) t -= 0.5 * j * (j - 1) * E[(j - 2) * DJ];
                tk[k] = t;
            }
            const double r = kPi / pb.p;
            const double pref = pb.K * r * sqrt(r);
            sacc += pref * sk[0] * sk[1] * sk[2];
            tacc += pref * (tk[0] * sk[1] * sk[2] + sk[0] * tk[1] * sk[2] + sk[0] * sk[1] * tk[2]);
        }
        __syncthreads();
    }
    if (tid < NA * NB) {
        const double f = (A.sh1 == A.sh2) ? 0.5 : 1.0;
        const int64_t o = (int64_t)(A.c1 + tid / NB) * ld + A.c2 + tid % NB;
        Sacc[o] = f * sacc;
        Tacc[o] = f * tacc;
    }
}

void launch_st_pair(int la, int lb, const CPair *cp, int ncp, const PrimPair *pp, double *Sacc, double *Tacc, int ld,
                    hipStream_t st)
{
    if (ncp <= 0) return;
#define MD_ST(A_, B_)                                                                                    \
    if (la == A_ && lb == B_) {                                                                          \
        hipLaunchKernelGGL((st_pair<A_, B_>), dim3((unsigned)ncp), dim3(128), 0, st, cp, ncp, pp, Sacc, Tacc, ld); \
        return;                                                                                          \
    }
    MD_ST(0, 0) MD_ST(1, 0) MD_ST(1, 1) MD_ST(2, 0) MD_ST(2, 1) MD_ST(2, 2) MD_ST(3, 0) MD_ST(3, 1)
    MD_ST(3, 2) MD_ST(3, 3)
#undef MD_ST
}

// R^0_t(p, P - C) times K_ab (2 pi/p) q for one primitive pair and one charge
template <int L>
__device__ __forceinline__ void charge_r(const PrimPair &pb, double cx, double cy, double cz, double q,
                                         const double *__restrict__ btab, double *R)
{
    const double X = pb.P[0] - cx, Y = pb.P[1] - cy, Z = pb.P[2] - cz;
    const double p = pb.p;
    double F[L + 1], Fs[L + 1];
    boys_all<L>(p * (X * X + Y * Y + Z * Z), F, btab);
    double s = 2.0 * kPi / p * pb.K * q;
    const double m2p = -2.0 * p;
#pragma unroll
    for (int m = 0; m <= L; ++m) {
        Fs[m] = s * F[m];
        s *= m2p;
    }
    r_build<L, double>(Fs, X, Y, Z, R);
}

// out[y * stride + g * NH + t] = Hermite potential of pair g over the charges
// [y * cper, min(nchg, (y + 1) * cper)) (zeros for an empty range)
template <int L>
__global__ __launch_bounds__(64) void vh_kernel(const PrimPair *__restrict__ pp, int pbase, int npp,
                                                const double *__restrict__ chg, int nchg, int cper,
                                                const double *__restrict__ btab, double *__restrict__ out,
                                                int64_t stride)
{
    constexpr int NH = nherm(L);
    const int g = blockIdx.x * 64 + threadIdx.x;
    if (g >= npp) return;  // no cross-lane work below
    const PrimPair pb = pp[pbase + g];
    const int c0 = blockIdx.y * cper, c1 = min(nchg, c0 + cper);
    double acc[NH];
#pragma unroll
    for (int t = 0; t < NH; ++t) acc[t] = 0.0;
    for (int c = c0; c < c1; ++c) {
        const double *C = chg + 4 * c;
        double R[NH];
        charge_r<L>(pb, C[0], C[1], C[2], C[3], btab, R);
#pragma unroll
        for (int t = 0; t < NH; ++t) acc[t] += R[t];
    }
    double *o = out + (int64_t)blockIdx.y * stride + (int64_t)g * NH;
#pragma unroll
    for (int t = 0; t < NH; ++t) o[t] = acc[t];
}

// out[i] = sum over s = 0 .. ns-1 (in order) of part[s * n + i]
__global__ void split_reduce(const double *__restrict__ part, int ns, int64_t n, double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < ns; ++k) s += part[(int64_t)k * n + i];
    out[i] = s;
}

// part[(y * nchg + c) * 3 + k] = -sum over the pairs [y * gper, min(npp, (y+1) * gper))
// of sum_t Dh_t R_{t+1_k}, for charge c = the lane's; Dt holds (-1)^{|t|} Dh_t
// (the J-engine's ket sign).
template <int L>
__global__ __launch_bounds__(64) void vgrad_charge(const PrimPair *__restrict__ pp, int pbase, int npp, int gper,
                                                   const double *__restrict__ Dt, const double *__restrict__ chg,
                                                   int nchg, const double *__restrict__ btab,
                                                   double *__restrict__ part)
{
    constexpr int NH = nherm(L), NH1 = nherm(L + 1);
    const int c = blockIdx.x * 64 + threadIdx.x;
    if (c >= nchg) return;  // no cross-lane work below
    const double cx = chg[4 * c], cy = chg[4 * c + 1], cz = chg[4 * c + 2], q = chg[4 * c + 3];
    const int g0 = blockIdx.y * gper, g1 = min(npp, g0 + gper);
    double gk[3] = {0.0, 0.0, 0.0};
    for (int g = g0; g < g1; ++g) {
        const PrimPair pb = pp[pbase + g];
        double R[NH1];
        charge_r<L + 1>(pb, cx, cy, cz, q, btab, R);
        const double *dt = Dt + (int64_t)g * NH;
        static_for<0, NH>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            constexpr int tx = herm_t(t), ty = herm_u(t), tz = herm_v(t);
            constexpr double sg = ((tx + ty + tz) & 1) ? -1.0 : 1.0;
            const double d = sg * dt[t];
            gk[0] += d * R[herm_idx(tx + 1, ty, tz)];
            gk[1] += d * R[herm_idx(tx, ty + 1, tz)];
            gk[2] += d * R[herm_idx(tx, ty, tz + 1)];
        });
    }
    double *o = part + ((int64_t)blockIdx.y * nchg + c) * 3;
    for (int k = 0; k < 3; ++k) o[k] = -gk[k];
}

// out[i] += sum over splits s (in order) of part[s * 3 nchg + i]
__global__ void vgrad_charge_reduce(const double *__restrict__ part, int nsplit, int nchg, double *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * nchg) return;
    double s = out[i];
    for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * 3 * nchg + i];
    out[i] = s;
}

int potential_splits(int npp, int nchg, int L, int64_t cap_doubles)
{
    if (npp <= 0 || nchg <= 0) return 1;
    const int groups = (npp + 63) / 64;
    int s = std::max(1, std::min(64, (4096 + groups - 1) / groups));
    s = std::min(s, std::max(1, nchg / 32));
    const int64_t per = (int64_t)npp * nherm(L);
    s = (int)std::min<int64_t>(s, std::max<int64_t>(1, cap_doubles / per));
    return s;
}

bool launch_vh(int L, const PrimPair *pp, int pbase, int npp, const double *chg, int nchg, const double *btab,
               double *Vh, double *part, int nsplit, hipStream_t st)
{
    if (npp <= 0) return true;
    if (nsplit < 1) nsplit = 1;
    const int cper = nsplit == 1 ? std::max(nchg, 1) : (nchg + nsplit - 1) / nsplit;
    const int64_t stride = (int64_t)npp * nherm(L);
    double *out = nsplit == 1 ? Vh : part;
    bool done = false;
    static_for<0, 8>([&](auto lc) {
        constexpr int Lc = decltype(lc)::value;
        if (!done && L == Lc) {
            hipLaunchKernelGGL((vh_kernel<Lc>), dim3((npp + 63) / 64, nsplit), dim3(64), 0, st, pp, pbase, npp, chg,
                               nchg, cper, btab, out, stride);
            done = true;
        }
    });
    if (done && nsplit > 1)
        hipLaunchKernelGGL(split_reduce, dim3((unsigned)((stride + 255) / 256)), dim3(256), 0, st, part, nsplit,
                           stride, Vh);
    return done;
}

bool launch_vgrad_charge(int L, const PrimPair *pp, int pbase, int npp, const double *Dt, const double *chg,
                         int nchg, const double *btab, double *part, int nsplit, double *gchg, hipStream_t st)
{
    if (npp <= 0 || nchg <= 0) return true;
    if (nsplit < 1) nsplit = 1;
    const int gper = (npp + nsplit - 1) / nsplit;
    bool done = false;
    static_for<0, 7>([&](auto lc) {
        constexpr int Lc = decltype(lc)::value;
        if (!done && L == Lc) {
            hipLaunchKernelGGL((vgrad_charge<Lc>), dim3((nchg + 63) / 64, nsplit), dim3(64), 0, st, pp, pbase, npp,
                               gper, Dt, chg, nchg, btab, part);
            hipLaunchKernelGGL(vgrad_charge_reduce, dim3((3 * nchg + 255) / 256), dim3(256), 0, st, part, nsplit,
                               nchg, gchg);
            done = true;
        }
    });
    return done;
}

}  // namespace md
