// jeng_reg.hpp -- J-engine step 2 for high total Hermite order with every
// operand in registers: one lane per bra primitive pair, kets wave-uniform.
// R^0_N is never stored: each entry is formed from the closed form
//   R^0_{tuv} = sum_{a,b,c} C_t^a C_u^b C_v^c X^{t-2a} Y^{u-2b} Z^{v-2c} G_{t+u+v-a-b-c}
// (G_n = pref (-2 alpha)^n F_n; same values as eq. R_recursion) and used at
// once for every (P, Q) with P + Q = N:  Jh_P += R_N Dt_Q   (eq. j_formula).
#pragma once
#include "kern_args.hpp"
#include "md_device.hpp"
#include "queue.hpp"

namespace md {

__host__ __device__ constexpr double hcoef(int t, int a)
{
    // t! / (a! (t-2a)! 2^a)
    double v = 1.0;
    for (int k = 0; k < a; ++k) v = v * (double)((t - 2 * k) * (t - 2 * k - 1)) / (2.0 * (k + 1));
    return v;
}

// dq: the ket's Hermite density, in registers or (large ket orders) read at
// each use through the wave-uniform pointer into HBM; SCALE multiplies entry Q
// by rp[|Q|] at use (single-precision form).
template <int LX, int LY, bool SCALE, typename T>
__device__ __forceinline__ void jeng_quartet_stream(const T *G, const T *px, const T *py,
                                                    const T *pz, const T *__restrict__ dq, const T *rp, T *Jh)
{
    constexpr int L = LX + LY;
    static_for<0, nherm(L)>([&](auto Nc) {
        constexpr int N = decltype(Nc)::value;
        constexpr int t = herm_t(N), u = herm_u(N), v = herm_v(N);
        T r = T(0);
        static_for<0, t / 2 + 1>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            static_for<0, u / 2 + 1>([&](auto bc) {
                constexpr int b = decltype(bc)::value;
                T rz = T(0);
                static_for<0, v / 2 + 1>([&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    rz += T(hcoef(v, c)) * pz[v - 2 * c] * G[t + u + v - a - b - c];
                });
                r += T(hcoef(t, a) * hcoef(u, b)) * px[t - 2 * a] * py[u - 2 * b] * rz;
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
                        constexpr int Q = herm_idx(t - p1, u - p2, v - p3);
                        if constexpr (SCALE)
                            Jh[herm_idx(p1, p2, p3)] += r * (dq[Q] * rp[(t - p1) + (u - p2) + (v - p3)]);
                        else
                            Jh[herm_idx(p1, p2, p3)] += r * dq[Q];
                    }
                });
            });
        });
    });
}

// Mixed mode: tile (wavefront of bra pairs, ket pair j) as in jeng_small;
// single-precision tiles are summed per ket pair and added in double.
template <int LX, int LY, typename T>
__device__ __forceinline__ void jeng_reg_run(const JArgs &a, int blk_x, int blk_y)
{
    constexpr int L = LX + LY, NX = nherm(LX), NY = nherm(LY);
    constexpr bool F32 = sizeof(T) == 4;
    constexpr bool DQMEM = NY > 20;  // ket density read at use instead of held in registers
    const int g = blk_x * 64 + threadIdx.x;
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
    double qmax = qi, Qw = Qi;
    for (int off = 32; off > 0; off >>= 1) {
        nvmax = max(nvmax, __shfl_xor(nvmax, off));
        qmax = fmax(qmax, __shfl_xor(qmax, off));
        Qw = fmax(Qw, __shfl_xor(Qw, off));
    }
    nvmax = __builtin_amdgcn_readfirstlane(nvmax);
    {
        const uint64_t bq = __double_as_longlong(qmax);
        const uint32_t lo32 = __builtin_amdgcn_readfirstlane((uint32_t)bq);
        const uint32_t hi32 = __builtin_amdgcn_readfirstlane((uint32_t)(bq >> 32));
        qmax = __longlong_as_double(((uint64_t)hi32 << 32) | lo32);
    }
    const int j0 = blk_y * a.kchunk;
    const int j1 = min(min(a.nket, j0 + a.kchunk), nvmax);

    const T *__restrict__ Dt = pick<T>(a.Dt, a.Dtf);
    T Jt[NX];
    double Jh[F32 ? NX : 1];
#pragma unroll
    for (int i = 0; i < NX; ++i) Jt[i] = T(0);
#pragma unroll
    for (int i = 0; i < (F32 ? NX : 1); ++i) Jh[i] = 0.0;
    for (int j = j0; j < j1; ++j) {
        if (a.mode && (Qw * a.QDket[j] >= a.tau_mix) != (a.mode == 1)) continue;
        if (a.tau_dens > 0.0 && Qw * a.QDket[j] < a.tau_dens) continue;  // density-weighted screen
        const CPair B = a.ket[j];
        for (int kp = 0; kp < B.np; ++kp) {
            const PrimPair pk = a.pp[B.poff + kp];
            if (qmax * pk.q < a.tau_prim) break;
            if (j < nv && qi * pk.q >= a.tau_prim) {
                T G[L + 1], px[L + 1], py[L + 1], pz[L + 1], Xt, Yt, Zt;
                T rp[LY + 1];
                if constexpr (F32) {  // scaled single-precision form (md_device.hpp)
                    float r;
                    quartet_fs_scaled<L>(pb, pk, a.boys, G, Xt, Yt, Zt, r, a.om2);
                    powers<LY>(r, rp);
                } else {
                    quartet_fs<L, T>(pb, pk, a.boys, G, Xt, Yt, Zt, a.om2);
                }
                powers<L>(Xt, px);
                powers<L>(Yt, py);
                powers<L>(Zt, pz);
                const T *__restrict__ dt = Dt + (int64_t)(B.poff + kp - a.dt_base) * NY;
                if constexpr (DQMEM) {
                    jeng_quartet_stream<LX, LY, F32, T>(G, px, py, pz, dt, rp, Jt);
                } else {
                    T dq[NY];
                    static_for<0, NY>([&](auto qc) {
                        constexpr int k = decltype(qc)::value;
                        if constexpr (F32)
                            dq[k] = dt[k] * rp[herm_t(k) + herm_u(k) + herm_v(k)];
                        else
                            dq[k] = dt[k];
                    });
                    jeng_quartet_stream<LX, LY, false, T>(G, px, py, pz, dq, rp, Jt);
                }
            }
        }
        if constexpr (F32) {
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                Jh[i] += (double)Jt[i];
                Jt[i] = T(0);
            }
        }
    }
    if (valid && (j1 > j0 || a.jh_part > 0)) {
        // scaled form: Jh_P = K_ab (2p)^{|P|/2} times the single-precision sum
        double cw[LX + 1];
        cw[0] = pb.K;
        const double c = sqrt(2.0 * pb.p);
#pragma unroll
        for (int k = 1; k <= LX; ++k) cw[k] = cw[k - 1] * c;
        static_for<0, NX>([&](auto pc) {
            constexpr int P = decltype(pc)::value;
            double v;
            if constexpr (F32) v = Jh[P] * cw[herm_t(P) + herm_u(P) + herm_v(P)]; else v = Jt[P];
            if (a.jh_part > 0)
                a.Jh[(int64_t)blk_y * a.jh_part + (int64_t)g * NX + P] = v;
            else
                unsafeAtomicAdd(&a.Jh[(int64_t)g * NX + P], v);
        });
    }
}

template <int LX, int LY, typename T>
__global__ __launch_bounds__(64) void jeng_reg(JArgs a)
{
    jeng_reg_run<LX, LY, T>(a, blockIdx.x, blockIdx.y);
}

// batch form: workgroup b runs block (items[b].y, items[b].z) of the
// launch whose arguments are tab[items[b].x]
template <int LX, int LY, typename T>
__global__ __launch_bounds__(64) void jeng_reg_q(const JArgs *__restrict__ tab, const int4 *__restrict__ items)
{
    const int4 it = items[blockIdx.x];
    JArgs a = tab[it.x];
    globalize(a);
    jeng_reg_run<LX, LY, T>(a, it.y, it.z);
}

// register J-engine is used where its live set (Hermite J, Boys values,
// coordinate powers and, up to 20 entries, the Hermite density) stays within
// about 115 doubles
__host__ __device__ constexpr bool jeng_reg_ok(int lx, int ly)
{
    return lx + ly >= 6 && nherm(lx) + 4 * (lx + ly + 1) + (nherm(ly) <= 20 ? nherm(ly) : 0) <= 116;
}

// The queue forms are instantiated in translation units of their own
// (jeng_reg_q_*.hip), which compile in parallel with the direct ones.
QueueLaunchFn jeng_reg_queue_fn_0(int lx, int ly, bool fp32);
QueueLaunchFn jeng_reg_queue_fn_1(int lx, int ly, bool fp32);
QueueLaunchFn jeng_reg_queue_fn_2(int lx, int ly, bool fp32);
QueueLaunchFn jeng_reg_queue_fn_3(int lx, int ly, bool fp32);
inline QueueLaunchFn jeng_reg_queue_fn(int lx, int ly, bool fp32)
{
    QueueLaunchFn f = jeng_reg_queue_fn_0(lx, ly, fp32);
    if (!f) f = jeng_reg_queue_fn_1(lx, ly, fp32);
    if (!f) f = jeng_reg_queue_fn_2(lx, ly, fp32);
    if (!f) f = jeng_reg_queue_fn_3(lx, ly, fp32);
    return f;
}

template <int LX, int LY>
void jeng_reg_launch_t(const JArgs &a, bool fp32, hipStream_t st)
{
    const int nch = (a.nket + a.kchunk - 1) / a.kchunk;
    if (a.nbp <= 0 || nch <= 0) return;
    dim3 grid((a.nbp + 63) / 64, nch);
    if (queue_sink()) {  // a batch plan: a wavefront of bra pairs against one ket chunk per block
        queue_record(jeng_reg_queue_fn(LX, LY, fp32), a, (int)grid.x, nch,
                     (double)(a.kchunk < a.nket ? a.kchunk : a.nket), "jeng_reg");
        return;
    }
    if (fp32)
        hipLaunchKernelGGL((jeng_reg<LX, LY, float>), grid, dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL((jeng_reg<LX, LY, double>), grid, dim3(64), 0, st, a);
}

}  // namespace md
