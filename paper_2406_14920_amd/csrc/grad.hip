// grad.hip -- Coulomb part of the nuclear gradient, the final per-atom sum
// and the energy E = 1/2 tr(PJ) - 1/4 tr(PK).
//
// Coulomb part (SI eqs. si_dE_J, si_dj_formula): with the Hermite J of order
// LX+1 of every bra primitive pair,
//     Jh_P = sum_kets sum_Q R_{P+Q} Dt_Q,    P in H(LX+1)
// (the J-engine called with the bra order raised by one), the bra centres
// of each unordered pair ab (f = 2 for distinct shells) get
//     dE_J/dA_k = f sum_{ab} P_ab sum_t Ed^{A,k}_t Jh_t,
//     dE_J/dA_k + dE_J/dB_k = f sum_{ab} P_ab sum_t E_t Jh_{t+1_k}
// (derivative coefficients as in grad.hpp).  Every pair is the bra once, so
// the ket centres are covered when their pair is the bra.
#include "grad.hpp"
#include "kern_args.hpp"
#include "launch.hpp"
#include "md_device.hpp"
#include "wave_r.hpp"

namespace md {

template <int LA, int LB>
__global__ __launch_bounds__(64) void jgrad_pair(JGArgs g)
{
    constexpr int NA = ncart(LA), NB = ncart(LB), NAB = NA * NB, LAB = LA + LB;
    constexpr int NX1 = nherm(LAB + 1);
    constexpr int EBJ = LAB + 2, EBI = (LB + 1) * EBJ, EBD = (LA + 2) * EBI;
    __shared__ double sE[3 * EBD];
    const int c = blockIdx.x;
    if (c >= g.ncp) return;
    const CPair A = g.cp[c];
    const int tid = threadIdx.x;
    const double f = (A.sh1 == A.sh2) ? 1.0 : 2.0;
    double gA[3] = {0.0, 0.0, 0.0}, gS[3] = {0.0, 0.0, 0.0};
    for (int ip = 0; ip < A.np; ++ip) {
        const PrimPair pb = g.pp[A.poff + ip];
        if (tid < 3) {
            const double pa = tid == 0 ? pb.PA[0] : (tid == 1 ? pb.PA[1] : pb.PA[2]);
            const double pbb = tid == 0 ? pb.PB[0] : (tid == 1 ? pb.PB[1] : pb.PB[2]);
            etab_lds<LA + 1, LB>(pa, pbb, pb.o2p, sE + tid * EBD);
        }
        __syncthreads();
        const double *jh = g.Jh1 + (int64_t)(A.poff + ip - g.jh_base) * NX1;
        const double a2 = 2.0 * pb.a;
        const double *Ex = sE, *Ey = sE + EBD, *Ez = sE + 2 * EBD;
        for (int ab = tid; ab < NAB; ab += 64) {
            const int i = ab / NB, j = ab % NB;
            int ax, ay, az, bx, by, bz;
            cart_rt(LA, i, ax, ay, az);
            cart_rt(LB, j, bx, by, bz);
            const double w = f * g.D[(int64_t)(A.c1 + i) * g.ld + A.c2 + j];
            for (int k = 0; k < 3; ++k) {
                double s = 0.0;
                for (int tx = 0; tx <= ax + bx + (k == 0); ++tx) {
                    const double fx = k == 0 ? dcoef(Ex, EBI, EBJ, ax, bx, tx, a2) : Ex[ax * EBI + bx * EBJ + tx];
                    for (int ty = 0; ty <= ay + by + (k == 1); ++ty) {
                        const double fy = k == 1 ? dcoef(Ey, EBI, EBJ, ay, by, ty, a2) : Ey[ay * EBI + by * EBJ + ty];
                        for (int tz = 0; tz <= az + bz + (k == 2); ++tz) {
                            const double fz = k == 2 ? dcoef(Ez, EBI, EBJ, az, bz, tz, a2) : Ez[az * EBI + bz * EBJ + tz];
                            s += fx * fy * fz * jh[herm_idx_rt(tx, ty, tz)];
                        }
                    }
                }
                gA[k] += w * s;
            }
            for (int tx = 0; tx <= ax + bx; ++tx)
                for (int ty = 0; ty <= ay + by; ++ty)
                    for (int tz = 0; tz <= az + bz; ++tz) {
                        const double e = w * Ex[ax * EBI + bx * EBJ + tx] * Ey[ay * EBI + by * EBJ + ty] *
                                         Ez[az * EBI + bz * EBJ + tz];
                        gS[0] += e * jh[herm_idx_rt(tx + 1, ty, tz)];
                        gS[1] += e * jh[herm_idx_rt(tx, ty + 1, tz)];
                        gS[2] += e * jh[herm_idx_rt(tx, ty, tz + 1)];
                    }
        }
        __syncthreads();
    }
    double v[6] = {gA[0], gA[1], gA[2], gS[0], gS[1], gS[2]};
#pragma unroll
    for (int q = 0; q < 6; ++q)
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off);
    if (tid == 0) {
        for (int k = 0; k < 3; ++k) {
            g.pg[(int64_t)c * 6 + k] = v[k];
            g.pg[(int64_t)c * 6 + 3 + k] = v[3 + k] - v[k];
        }
    }
}

// grad[atom][k] = the exchange workgroup partials and the contracted pairs'
// Coulomb centre terms, summed in a fixed order in two steps: workgroup ch
// sums the rows of chunk ch (kGradRowsK partial rows, or kGradRowsP pairs)
// column by column into part[ch], then one thread per column adds the
// chunks in order.  Repeated calls give identical bits.
constexpr int kGradRowsK = 256, kGradRowsP = 256;

int grad_reduce_chunks(int ncp, int64_t nkblocks)
{
    return (int)((nkblocks + kGradRowsK - 1) / kGradRowsK) + (ncp + kGradRowsP - 1) / kGradRowsP;
}

__global__ __launch_bounds__(256) void grad_chunk_sums(const CPair *__restrict__ cp, int ncp,
                                                       const double *__restrict__ pg,
                                                       const double *__restrict__ kpart, int64_t nkblocks,
                                                       int natom, int nkc, double *__restrict__ part)
{
    const int n3 = 3 * natom, ch = blockIdx.x;
    for (int col = threadIdx.x; col < n3; col += blockDim.x) {
        double s = 0.0;
        if (ch < nkc) {
            const int64_t b0 = (int64_t)ch * kGradRowsK;
            const int64_t b1 = b0 + kGradRowsK < nkblocks ? b0 + kGradRowsK : nkblocks;
            for (int64_t b = b0; b < b1; ++b) s += kpart[b * n3 + col];
        } else {
            const int atom = col / 3, k = col % 3;
            const int p0 = (ch - nkc) * kGradRowsP, p1 = p0 + kGradRowsP < ncp ? p0 + kGradRowsP : ncp;
            for (int p = p0; p < p1; ++p) {
                const CPair c = cp[p];
                if (c.at1 == atom) s += pg[(int64_t)p * 6 + k];
                if (c.at2 == atom) s += pg[(int64_t)p * 6 + 3 + k];
            }
        }
        part[(int64_t)ch * n3 + col] = s;
    }
}

__global__ void grad_chunk_final(const double *__restrict__ part, int nch, int n3, double *__restrict__ grad)
{
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= n3) return;
    double s = 0.0;
    for (int ch = 0; ch < nch; ++ch) s += part[(int64_t)ch * n3 + col];
    grad[col] = s;
}

// E = sum_ij P_ij (J_ij / 2 - K_ij / 4), one workgroup, fixed-order tree.
__global__ __launch_bounds__(256) void energy_kernel(const double *__restrict__ P, const double *__restrict__ J,
                                                     const double *__restrict__ K, int64_t n2, double *E)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n2; i += 256) acc += P[i] * (0.5 * J[i] - 0.25 * K[i]);
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *E = s[0];
}

void launch_jgrad(int la, int lb, const JGArgs &g, hipStream_t st)
{
    if (g.ncp <= 0) return;
#define MD_JG(A_, B_)                                                                    \
    if (la == A_ && lb == B_) {                                                          \
        hipLaunchKernelGGL((jgrad_pair<A_, B_>), dim3((unsigned)g.ncp), dim3(64), 0, st, g); \
        return;                                                                          \
    }
    MD_JG(0, 0) MD_JG(1, 0) MD_JG(1, 1) MD_JG(2, 0) MD_JG(2, 1) MD_JG(2, 2) MD_JG(3, 0) MD_JG(3, 1)
    MD_JG(3, 2) MD_JG(3, 3)
#undef MD_JG
}

void launch_grad_reduce(const CPair *cp, int ncp, const double *pg, const double *kpart, int64_t nkblocks,
                        int natom, double *grad, double *part, hipStream_t st)
{
    const int n = 3 * natom;
    const int nkc = (int)((nkblocks + kGradRowsK - 1) / kGradRowsK);
    const int nch = grad_reduce_chunks(ncp, nkblocks);
    if (nch > 0)
        hipLaunchKernelGGL(grad_chunk_sums, dim3((unsigned)nch), dim3(256), 0, st, cp, ncp, pg, kpart, nkblocks,
                           natom, nkc, part);
    hipLaunchKernelGGL(grad_chunk_final, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, part, nch, n, grad);
}

void launch_energy(const double *P, const double *J, const double *K, int64_t n2, double *E, hipStream_t st)
{
    hipLaunchKernelGGL(energy_kernel, dim3(1), dim3(256), 0, st, P, J, K, n2, E);
}

}  // namespace md
