// count.hip -- counts the primitive quartets the J and K kernels evaluate,
// with exactly their screening loops (sorted pair lists, early exits), so the
// algorithmic FLOP model can be applied per launch.
#include "kern_args.hpp"
#include "launch.hpp"

namespace md {

__global__ void k_count(KArgs a, unsigned long long *out)
{
    int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long n = 0;
    if (w < a.nwork) {
        int lo = 0, hi = a.nbra;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (a.prefix[mid] <= w) lo = mid; else hi = mid;
        }
        const CPair A = a.bra[lo];
        const CPair B = a.ket[(int)(w - a.prefix[lo])];
        const double qk0 = a.pp[B.poff].q;
        for (int ip = 0; ip < A.np; ++ip) {
            const double qb = a.pp[A.poff + ip].q;
            if (qb * qk0 < a.tau_prim) break;
            for (int kp = 0; kp < B.np; ++kp) {
                if (qb * a.pp[B.poff + kp].q < a.tau_prim) break;
                ++n;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off);
    if ((threadIdx.x & 63) == 0 && n) atomicAdd(out, n);
}

__global__ void j_count(JArgs a, unsigned long long *out)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long n = 0;
    if (g < a.nbp) {
        const double qi = a.pp[a.pbase + g].q;
        const double Qi = a.Qbra[a.owner[g]];
        for (int j = 0; j < a.nket; ++j) {
            if (Qi * a.Qket[j] < a.tau) break;
            const CPair B = a.ket[j];
            for (int kp = 0; kp < B.np; ++kp) {
                if (qi * a.pp[B.poff + kp].q < a.tau_prim) break;
                ++n;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off);
    if ((threadIdx.x & 63) == 0 && n) atomicAdd(out, n);
}

void launch_k_count(const KArgs &a, unsigned long long *out, hipStream_t st)
{
    if (a.nwork <= 0) return;
    hipLaunchKernelGGL(k_count, dim3((unsigned)((a.nwork + 255) / 256)), dim3(256), 0, st, a, out);
}

void launch_j_count(const JArgs &a, unsigned long long *out, hipStream_t st)
{
    if (a.nbp <= 0 || a.nket <= 0) return;
    hipLaunchKernelGGL(j_count, dim3((unsigned)((a.nbp + 255) / 256)), dim3(256), 0, st, a, out);
}

}  // namespace md
