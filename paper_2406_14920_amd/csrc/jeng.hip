// jeng.hip -- Coulomb matrix by the J-engine (eq. j_formula) in three steps:
//   1. Hermite density of every ket primitive pair
//        Dt_Q = (-1)^{|Q|} f sum_{cd} E^{cd}_Q D_cd                (f = 2 for c != d shells)
//   2. Hermite J of every bra primitive pair
//        Jh_P = sum_{kets} sum_Q R_{P+Q} Dt_Q
//      (R carries the prefactor of eq. eri_formula and both pair factors K)
//   3. back to Cartesian: J_ab = sum_P E^{ab}_P Jh_P, written as one
//      triangle of the accumulator (J = Jacc + Jacc^T).
// Step 2 depends only on the total bra / ket Hermite orders (LX, LY); low
// orders keep R in registers (one lane per bra primitive pair), high orders
// build R in LDS with one wavefront per bra primitive pair.
#include "kern_args.hpp"
#include "md_device.hpp"
#include "queue.hpp"
#include "wave_r.hpp"

namespace md {

// ---------------------------------------------------------------------------
// 1. Hermite density: one workgroup per contracted ket pair
// ---------------------------------------------------------------------------
template <int LC, int LD>
__global__ __launch_bounds__(128) void hermite_density(const CPair *__restrict__ cp, int ncp,
                                                       const PrimPair *__restrict__ pp,
                                                       const double *__restrict__ D, int ld,
                                                       double *__restrict__ Dt, float *__restrict__ Dtf,
                                                       int dt_base)
{
    constexpr int NC = ncart(LC), ND = ncart(LD), LCD = LC + LD, NH = nherm(LCD);
    constexpr int EKD = (LC + 1) * (LD + 1) * (LCD + 1);
    __shared__ double sE[3 * EKD];
    __shared__ double sDb[NC * ND];
    const int c = blockIdx.x;
    if (c >= ncp) return;
    const CPair B = cp[c];
    const int tid = threadIdx.x;
    for (int o = tid; o < NC * ND; o += blockDim.x)
        sDb[o] = D[(int64_t)(B.c1 + o / ND) * ld + B.c2 + o % ND];
    const double f = (B.sh1 == B.sh2) ? 1.0 : 2.0;
    for (int kp = 0; kp < B.np; ++kp) {
        const PrimPair pk = pp[B.poff + kp];
        if (tid < 3) {
            const double pa = tid == 0 ? pk.PA[0] : (tid == 1 ? pk.PA[1] : pk.PA[2]);
            const double pbb = tid == 0 ? pk.PB[0] : (tid == 1 ? pk.PB[1] : pk.PB[2]);
            etab_lds<LC, LD>(pa, pbb, pk.o2p, sE + tid * EKD);
        }
        __syncthreads();
        for (int Q = tid; Q < NH; Q += blockDim.x) {
            const int code = c_herm.tuv[Q];
            const int qt = code & 0xff, qu = (code >> 8) & 0xff, qv = code >> 16;
            double acc = 0.0;
            for (int cd = 0; cd < NC * ND; ++cd) {
                int cx, cy, cz, dx, dy, dz;
                cart_rt(LC, cd / ND, cx, cy, cz);
                cart_rt(LD, cd % ND, dx, dy, dz);
                if (qt > cx + dx || qu > cy + dy || qv > cz + dz) continue;
                acc += sE[(cx * (LD + 1) + dx) * (LCD + 1) + qt] *
                       sE[EKD + (cy * (LD + 1) + dy) * (LCD + 1) + qu] *
                       sE[2 * EKD + (cz * (LD + 1) + dz) * (LCD + 1) + qv] * sDb[cd];
            }
            const double sg = ((qt + qu + qv) & 1) ? -1.0 : 1.0;
            const int64_t o = (int64_t)(B.poff + kp - dt_base) * NH + Q;
            Dt[o] = sg * f * acc;
            if (Dtf) {  // scaled single-precision form: K_cd Dt_Q (2q)^{|Q|/2}
                double sc = pk.K;
                const double c = sqrt(2.0 * pk.p);
                for (int k = 0; k < qt + qu + qv; ++k) sc *= c;
                Dtf[o] = (float)(sg * f * acc * sc);
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ int wave_max(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ double uniform_d(double v)
{
    const uint64_t b = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double(((uint64_t)hi << 32) | lo);
}

// number of class-Y kets j with Qi * Q_j >= tau (Q sorted descending)
__device__ __forceinline__ int count_kets(const double *__restrict__ Q, int n, double Qi, double tau)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (Qi * Q[mid] >= tau) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// 2a. Hermite J, registers: one lane per bra primitive pair
// ---------------------------------------------------------------------------
// In the mixed mode the precision tile is (wavefront of bra pairs, ket pair
// j): double precision when max_wave(Q_ab) Q_cd max|D_cd| reaches the
// threshold.  Single-precision tiles are summed per ket pair in T and added to
// a double-precision accumulator.
template <int LX, int LY, typename T>
__device__ __forceinline__ void jeng_small_run(const JArgs &a, int blk_x, int blk_y)
{
    constexpr int L = LX + LY, NX = nherm(LX), NY = nherm(LY);
    constexpr bool F32 = sizeof(T) == 4;
    const int g = blk_x * 64 + threadIdx.x;
    const bool valid = g < a.nbp;
    const int gi = valid ? g : a.nbp - 1;
    const PrimPair pb = a.pp[a.pbase + gi];
    const double Qi = valid ? a.Qbra[a.owner[gi]] : 0.0;
    const double qi = valid ? pb.q : 0.0;
    const int nv = valid ? count_kets(a.Qket, a.nket, Qi, a.tau) : 0;
    const int nvmax = __builtin_amdgcn_readfirstlane(wave_max(nv));
    const double qmax = uniform_d(wave_max(qi));
    const double Qw = (a.mode || a.tau_dens > 0.0) ? uniform_d(wave_max(Qi)) : 0.0;
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
                T Fs[L + 1], X, Y, Z;
                T rp[LY + 1];
                if constexpr (F32) {
                    float r;
                    quartet_fs_scaled<L>(pb, pk, a.boys, Fs, X, Y, Z, r, a.om2);
                    powers<LY>(r, rp);
                } else {
                    quartet_fs<L, T>(pb, pk, a.boys, Fs, X, Y, Z, a.om2);
                }
                T R[nherm(L)];
                r_build<L, T>(Fs, X, Y, Z, R);
                const T *dt = Dt + (int64_t)(B.poff + kp - a.dt_base) * NY;
                T dq[NY];
                static_for<0, NY>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    if constexpr (F32)
                        dq[q] = dt[q] * rp[herm_t(q) + herm_u(q) + herm_v(q)];
                    else
                        dq[q] = dt[q];
                });
                static_for<0, NX>([&](auto pc) {
                    constexpr int P = decltype(pc)::value;
                    constexpr int tp = herm_t(P), up = herm_u(P), vp = herm_v(P);
                    T acc = Jt[P];
                    static_for<0, NY>([&](auto qc) {
                        constexpr int Q = decltype(qc)::value;
                        acc += R[herm_idx(tp + herm_t(Q), up + herm_u(Q), vp + herm_v(Q))] * dq[Q];
                    });
                    Jt[P] = acc;
                });
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
__global__ __launch_bounds__(64) void jeng_small(JArgs a)
{
    jeng_small_run<LX, LY, T>(a, blockIdx.x, blockIdx.y);
}

// batch form: workgroup b runs block (items[b].y, items[b].z) of the
// launch whose arguments are tab[items[b].x]
template <int LX, int LY, typename T>
__global__ __launch_bounds__(64) void jeng_small_q(const JArgs *__restrict__ tab, const int4 *__restrict__ items)
{
    const int4 it = items[blockIdx.x];
    JArgs a = tab[it.x];
    globalize(a);
    jeng_small_run<LX, LY, T>(a, it.y, it.z);
}

// ---------------------------------------------------------------------------
// 2b. Hermite J, LDS: one wavefront per (bra primitive pair, ket chunk)
// ---------------------------------------------------------------------------
// Mixed mode: the tile is (bra primitive pair, ket pair j).
template <int LX, int LY, typename T>
__device__ __forceinline__ void jeng_wave_run(const JArgs &a, int blk_x, int blk_y)
{
    constexpr int L = LX + LY, L1 = L + 1, NX = nherm(LX), NY = nherm(LY);
    __shared__ T sR0[L1 * L1 * L1];
    __shared__ T sF[L + 1];
    __shared__ T sH[HPolyDims<L>::N];
    __shared__ int sHerm[nherm(L)];
    __shared__ T sDq[NY];  // single precision: r^|Q| times the scaled Hermite density
    const int lane = threadIdx.x;
    herm_table_lds(sHerm, nherm(L), lane);
    // per-lane R^0 term plan (L <= 9), visible after the first barrier
    __shared__ uint32_t sPlan[R0Plan<L, T>::OK ? R0Plan<L, T>::NT * 64 : 1];
    R0Plan<L, T> r0p;
    r0p.code = sPlan;
    if constexpr (R0Plan<L, T>::OK) r0_plan_build<L, T>(r0p, lane);
    const int g = blk_x;
    const PrimPair pb = a.pp[a.pbase + g];
    const double Qi = a.Qbra[a.owner[g]];
    const double qi = pb.q;
    const int nv = count_kets(a.Qket, a.nket, Qi, a.tau);
    const int j0 = blk_y * a.kchunk;
    const int j1 = min(min(a.nket, j0 + a.kchunk), nv);
    if (j1 <= j0 && a.jh_part == 0) return;  // (per-chunk stores still write their zeros)

    // lane owns P = lane and P = lane + 64
    int pof[2];
    bool own[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int P = lane + 64 * r;
        own[r] = P < NX;
        const int code = c_herm.tuv[own[r] ? P : 0];
        pof[r] = ((code & 0xff) * L1 + ((code >> 8) & 0xff)) * L1 + (code >> 16);
    }
    const T *__restrict__ Dt = pick<T>(a.Dt, a.Dtf);
    double acc[2] = {0.0, 0.0};
    for (int j = j0; j < j1; ++j) {
        if (a.mode && (Qi * a.QDket[j] >= a.tau_mix) != (a.mode == 1)) continue;
        if (a.tau_dens > 0.0 && Qi * a.QDket[j] < a.tau_dens) continue;  // density-weighted screen
        const CPair B = a.ket[j];
        PairLite pk = pair_lite(a.pp + B.poff);
        for (int kp = 0; kp < B.np; ++kp) {
            if (qi * pk.q < a.tau_prim) break;
            const PairLite pk_next = pair_lite(a.pp + B.poff + (kp + 1 < B.np ? kp + 1 : kp));
            const QuartetGeo geo = quartet_geo(pb, pk, a.om2);
            wave_boys<L, T>(geo, a.boys, sF, lane);
            wave_hpoly<L, T>(geo, sH, lane);
            const T *dt = Dt + (int64_t)(B.poff + kp - a.dt_base) * NY;
            if constexpr (sizeof(T) == 4) {
                for (int Q = lane; Q < NY; Q += 64) {
                    const int code = c_herm.tuv[Q];
                    const int n = (code & 0xff) + ((code >> 8) & 0xff) + (code >> 16);
                    float w = dt[Q];
                    const float r = (float)geo.r;
                    for (int k = 0; k < n; ++k) w *= r;
                    sDq[Q] = w;
                }
                dt = sDq;
            }
            __syncthreads();
            if constexpr (R0Plan<L, T>::OK)
                wave_r0h_plan<L, T>(r0p, sF, sH, sR0, lane);
            else
                wave_r0h<L, T>(sF, sH, sHerm, sR0, lane);
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                if (!own[r]) continue;
                const T *Rb = sR0 + pof[r];
                T s = T(0);
                static_for<0, NY>([&](auto qc) {
                    constexpr int Q = decltype(qc)::value;
                    constexpr int qo = (herm_t(Q) * L1 + herm_u(Q)) * L1 + herm_v(Q);
                    s += Rb[qo] * dt[Q];
                });
                acc[r] += (double)s;
            }
            __syncthreads();
            pk = pk_next;
        }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
        if (own[r]) {
            double v = acc[r];
            if constexpr (sizeof(T) == 4) {  // K_ab (2p)^{|P|/2} of the scaled form
                const int code = c_herm.tuv[lane + 64 * r];
                const int n = (code & 0xff) + ((code >> 8) & 0xff) + (code >> 16);
                const double c = sqrt(2.0 * pb.p);
                v *= pb.K;
                for (int k = 0; k < n; ++k) v *= c;
            }
            if (a.jh_part > 0)
                a.Jh[(int64_t)blk_y * a.jh_part + (int64_t)g * NX + lane + 64 * r] = v;
            else
                unsafeAtomicAdd(&a.Jh[(int64_t)g * NX + lane + 64 * r], v);
        }
}

template <int LX, int LY, typename T>
__global__ __launch_bounds__(64) void jeng_wave(JArgs a)
{
    jeng_wave_run<LX, LY, T>(a, blockIdx.x, blockIdx.y);
}

// batch form: workgroup b runs block (items[b].y, items[b].z) of the
// launch whose arguments are tab[items[b].x]
template <int LX, int LY, typename T>
__global__ __launch_bounds__(64) void jeng_wave_q(const JArgs *__restrict__ tab, const int4 *__restrict__ items)
{
    const int4 it = items[blockIdx.x];
    JArgs a = tab[it.x];
    globalize(a);
    jeng_wave_run<LX, LY, T>(a, it.y, it.z);
}

// out[i] += sum over the chunks c = 0, 1, ... of part[c * stride + i], in that
// order (the gradient's Hermite J: repeatable sums with many ket chunks)
__global__ void jh_reduce(const double *__restrict__ part, int nch, int64_t stride, double *__restrict__ out,
                          int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = out[i];
    for (int c = 0; c < nch; ++c) s += part[(int64_t)c * stride + i];
    out[i] = s;
}

void launch_jh_reduce(const double *part, int nch, int64_t stride, double *out, int64_t n, hipStream_t st)
{
    if (n <= 0 || nch <= 0) return;
    hipLaunchKernelGGL(jh_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, nch, stride, out, n);
}

// ---------------------------------------------------------------------------
// 3. Hermite J -> Cartesian J accumulator: one workgroup per contracted pair
// ---------------------------------------------------------------------------
template <int LA, int LB>
__global__ __launch_bounds__(128) void hermite_to_cart(const CPair *__restrict__ cp, int ncp,
                                                       const PrimPair *__restrict__ pp,
                                                       const double *__restrict__ Jh, int jh_base,
                                                       double *__restrict__ Jacc, int ld)
{
    constexpr int NA = ncart(LA), NB = ncart(LB), LAB = LA + LB, NH = nherm(LAB);
    constexpr int EBD = (LA + 1) * (LB + 1) * (LAB + 1);
    __shared__ double sE[3 * EBD];
    const int c = blockIdx.x;
    if (c >= ncp) return;
    const CPair A = cp[c];
    const int tid = threadIdx.x;
    double acc = 0.0;
    int ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
    if (tid < NA * NB) {
        cart_rt(LA, tid / NB, ax, ay, az);
        cart_rt(LB, tid % NB, bx, by, bz);
    }
    for (int ip = 0; ip < A.np; ++ip) {
        const PrimPair pb = pp[A.poff + ip];
        if (tid < 3) {
            const double pa = tid == 0 ? pb.PA[0] : (tid == 1 ? pb.PA[1] : pb.PA[2]);
            const double pbb = tid == 0 ? pb.PB[0] : (tid == 1 ? pb.PB[1] : pb.PB[2]);
            etab_lds<LA, LB>(pa, pbb, pb.o2p, sE + tid * EBD);
        }
        __syncthreads();
        if (tid < NA * NB) {
            const double *jh = Jh + (int64_t)(A.poff + ip - jh_base) * NH;
            double s = 0.0;
            for (int tx = 0; tx <= ax + bx; ++tx)
                for (int ty = 0; ty <= ay + by; ++ty)
                    for (int tz = 0; tz <= az + bz; ++tz)
                        s += sE[(ax * (LB + 1) + bx) * (LAB + 1) + tx] *
                             sE[EBD + (ay * (LB + 1) + by) * (LAB + 1) + ty] *
                             sE[2 * EBD + (az * (LB + 1) + bz) * (LAB + 1) + tz] *
                             jh[herm_idx_rt(tx, ty, tz)];
            acc += s;
        }
        __syncthreads();
    }
    if (tid < NA * NB) {
        const double f = (A.sh1 == A.sh2) ? 0.5 : 1.0;
        Jacc[(int64_t)(A.c1 + tid / NB) * ld + A.c2 + tid % NB] = f * acc;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_hermite_density(int lc, int ld_, const CPair *cp, int ncp, const PrimPair *pp,
                            const double *D, int ldd, double *Dt, float *Dtf, int dt_base, hipStream_t st)
{
    if (ncp <= 0) return;
#define MD_HD(C_, D_)                                                                         \
    if (lc == C_ && ld_ == D_) {                                                             \
        hipLaunchKernelGGL((hermite_density<C_, D_>), dim3(ncp), dim3(128), 0, st, cp, ncp, pp, D, \
                           ldd, Dt, Dtf, dt_base);                                                \
        return;                                                                              \
    }
    MD_HD(0, 0) MD_HD(1, 0) MD_HD(1, 1) MD_HD(2, 0) MD_HD(2, 1) MD_HD(2, 2) MD_HD(3, 0) MD_HD(3, 1)
    MD_HD(3, 2) MD_HD(3, 3)
#undef MD_HD
}

void launch_hermite_to_cart(int la, int lb, const CPair *cp, int ncp, const PrimPair *pp,
                            const double *Jh, int jh_base, double *Jacc, int ld, hipStream_t st)
{
    if (ncp <= 0) return;
#define MD_HC(A_, B_)                                                                          \
    if (la == A_ && lb == B_) {                                                               \
        hipLaunchKernelGGL((hermite_to_cart<A_, B_>), dim3(ncp), dim3(128), 0, st, cp, ncp, pp, Jh, \
                           jh_base, Jacc, ld);                                                \
        return;                                                                               \
    }
    MD_HC(0, 0) MD_HC(1, 0) MD_HC(1, 1) MD_HC(2, 0) MD_HC(2, 1) MD_HC(2, 2) MD_HC(3, 0) MD_HC(3, 1)
    MD_HC(3, 2) MD_HC(3, 3)
#undef MD_HC
}

// total Hermite order at or below which the register path is used
constexpr int kJengRegMaxL = 5;

bool launch_jeng_reg_0(int lx, int ly, const JArgs &a, bool fp32, hipStream_t st);
bool launch_jeng_reg_1(int lx, int ly, const JArgs &a, bool fp32, hipStream_t st);
bool launch_jeng_reg_2(int lx, int ly, const JArgs &a, bool fp32, hipStream_t st);
bool launch_jeng_reg_3(int lx, int ly, const JArgs &a, bool fp32, hipStream_t st);

template <int LX, int LY, typename T>
void jeng_launch_t(const JArgs &a, hipStream_t st)
{
    constexpr bool f32 = sizeof(T) == 4;
    if (launch_jeng_reg_0(LX, LY, a, f32, st) || launch_jeng_reg_1(LX, LY, a, f32, st) ||
        launch_jeng_reg_2(LX, LY, a, f32, st) || launch_jeng_reg_3(LX, LY, a, f32, st))
        return;
    const int nch = (a.nket + a.kchunk - 1) / a.kchunk;
    if (a.nbp <= 0 || nch <= 0) return;
    constexpr bool SMALL = LX + LY <= kJengRegMaxL;
    const dim3 grid(SMALL ? (a.nbp + 63) / 64 : a.nbp, nch);
    if (queue_sink()) {  // a batch plan (builds only: bra order at most 6)
        QueueLaunchFn fn = nullptr;
        if constexpr (LX <= 6) {
            if constexpr (SMALL)
                fn = &queue_launch<JArgs, jeng_small_q<LX, LY, T>, 64>;
            else
                fn = &queue_launch<JArgs, jeng_wave_q<LX, LY, T>, 64>;
        }
        queue_record(fn, a, (int)grid.x, nch, (double)(a.kchunk < a.nket ? a.kchunk : a.nket),
                     SMALL ? "jeng_small" : "jeng_wave");
        return;
    }
    if constexpr (SMALL)
        hipLaunchKernelGGL((jeng_small<LX, LY, T>), grid, dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL((jeng_wave<LX, LY, T>), grid, dim3(64), 0, st, a);
}

// Bra orders up to 7 serve the gradient (the bra order raised by one), which
// runs in double precision only.
bool launch_jeng(int lx, int ly, const JArgs &a, bool fp32, hipStream_t st)
{
    bool done = false;
    if (fp32 && lx > 6) return false;
    static_for<0, 8>([&](auto xc) {
        constexpr int X = decltype(xc)::value;
        static_for<0, 7>([&](auto yc) {
            constexpr int Yv = decltype(yc)::value;
            if (!done && lx == X && ly == Yv) {
                if constexpr (X <= 6) {
                    if (fp32) jeng_launch_t<X, Yv, float>(a, st); else jeng_launch_t<X, Yv, double>(a, st);
                } else {
                    jeng_launch_t<X, Yv, double>(a, st);
                }
                done = true;
            }
        });
    });
    return done;
}

}  // namespace md
