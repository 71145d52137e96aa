// count.hip -- counts the primitive quartets the J and K kernels evaluate,
// with exactly their screening loops (sorted pair lists, early exits), so the
// algorithmic FLOP model can be applied per launch.
#include "kern_args.hpp"
#include "launch.hpp"
#include "md_device.hpp"

namespace md {

__global__ void k_count(KArgs a, unsigned long long *out)
{
    int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long n = 0;
    if (w < a.nwork) {
        const int row = k_find_row(a.prefix, a.nrows, w);
        const int2 rw = a.rows[row];
        const CPair A = a.bra[rw.x];
        const CPair B = a.ket[rw.y + (int)(w - a.prefix[row])];
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

// ---------------------------------------------------------------------------
// Single-precision share of a mixed-precision build, with the tile rule of
// each kernel family (md_device.hpp: mix_take).  out[0] += primitive
// quartets, out[1] += contracted quartets (or ket pairs for the J-engine).
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long prim_quartets(const KArgs &a, const CPair &A, const CPair &B)
{
    unsigned long long n = 0;
    const double qk0 = a.pp[B.poff].q;
    for (int ip = 0; ip < A.np; ++ip) {
        const double qb = a.pp[A.poff + ip].q;
        if (qb * qk0 < a.tau_prim) break;
        for (int kp = 0; kp < B.np; ++kp) {
            if (qb * a.pp[B.poff + kp].q < a.tau_prim) break;
            ++n;
        }
    }
    return n;
}

__device__ __forceinline__ void wave_add2(unsigned long long n, unsigned long long m, unsigned long long *out)
{
    for (int off = 32; off > 0; off >>= 1) {
        n += __shfl_xor(n, off);
        m += __shfl_xor(m, off);
    }
    if ((threadIdx.x & 63) == 0 && (n || m)) {
        atomicAdd(out, n);
        atomicAdd(out + 1, m);
    }
}

__global__ void k_count_mix(KArgs a, int kind, unsigned long long *out)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = w < a.nwork;
    int ib = 0, jk = 0;
    bool need = false;
    if (valid) {
        const int row = k_find_row(a.prefix, a.nrows, w);
        ib = a.rows[row].x;
        jk = a.rows[row].y + (int)(w - a.prefix[row]);
        need = a.Qbra[ib] * a.Qket[jk] * k_dens_bound(a.Pm, a.nsh, a.bra[ib], a.ket[jk]) >= a.tau_mix;
    }
    const bool tile_fp64 = kind == 0 ? (__ballot(need ? 1 : 0) != 0ull) : need;
    unsigned long long n = 0, m = 0;
    if (valid && !tile_fp64) {
        n = prim_quartets(a, a.bra[ib], a.ket[jk]);
        m = 1;
    }
    wave_add2(n, m, out);
}

__global__ __launch_bounds__(64) void k_count_mix_chunks(KArgs a, const int4 *__restrict__ chunks,
                                                          unsigned long long *out)
{
    const int4 ch = chunks[blockIdx.x];
    const int lane = (int)threadIdx.x;
    const bool valid = lane < ch.z;
    const int64_t wl = a.prefix[ch.x] + ch.y + (valid ? lane : 0);
    int r = ch.x;
    for (int k = 1; k < ch.w; ++k)
        if (a.prefix[ch.x + k] <= wl) r = ch.x + k;
    const int ib = a.rows[ch.x].x;
    const int jk = a.rows[r].y + (int)(wl - a.prefix[r]);
    const CPair A = a.bra[ib];
    const CPair B = a.ket[jk];
    const bool need = valid && a.Qbra[ib] * a.Qket[jk] * k_dens_bound(a.Pm, a.nsh, A, B) >= a.tau_mix;
    const bool tile_fp64 = __ballot(need ? 1 : 0) != 0ull;
    unsigned long long n = 0, m = 0;
    if (valid && !tile_fp64) {
        n = prim_quartets(a, A, B);
        m = 1;
    }
    wave_add2(n, m, out);
}

__global__ void j_count_mix(JArgs a, int per_bra, unsigned long long *out)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = g < a.nbp;
    const double Qi = valid ? a.Qbra[a.owner[g]] : 0.0;
    double Qw = Qi;
    if (!per_bra)
        for (int off = 32; off > 0; off >>= 1) Qw = fmax(Qw, __shfl_xor(Qw, off));
    unsigned long long n = 0, m = 0;
    if (valid) {
        const double qi = a.pp[a.pbase + g].q;
        for (int j = 0; j < a.nket; ++j) {
            if (Qi * a.Qket[j] < a.tau) break;
            if (Qw * a.QDket[j] >= a.tau_mix) continue;
            const CPair B = a.ket[j];
            ++m;
            for (int kp = 0; kp < B.np; ++kp) {
                if (qi * a.pp[B.poff + kp].q < a.tau_prim) break;
                ++n;
            }
        }
    }
    wave_add2(n, m, out);
}

void launch_k_count_mix(const KArgs &a, int kind, const int4 *chunks, int nchunks, unsigned long long *out,
                        hipStream_t st)
{
    if (a.nwork <= 0) return;
    if (kind == 2) {
        if (nchunks > 0)
            hipLaunchKernelGGL(k_count_mix_chunks, dim3((unsigned)nchunks), dim3(64), 0, st, a, chunks, out);
        return;
    }
    hipLaunchKernelGGL(k_count_mix, dim3((unsigned)((a.nwork + 255) / 256)), dim3(256), 0, st, a, kind, out);
}

void launch_j_count_mix(const JArgs &a, int per_bra, unsigned long long *out, hipStream_t st)
{
    if (a.nbp <= 0 || a.nket <= 0) return;
    hipLaunchKernelGGL(j_count_mix, dim3((unsigned)((a.nbp + 255) / 256)), dim3(256), 0, st, a, per_bra, out);
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
