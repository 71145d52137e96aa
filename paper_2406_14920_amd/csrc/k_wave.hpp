// k_wave.hpp -- exchange (K) for the highest angular classes (total L >= 7):
// one 64-lane workgroup evaluates one canonical contracted shell quartet at a
// time.  Per primitive quartet the lanes evaluate F_m and the coordinate
// powers, copy the bra and ket Hermite products of the two primitive pairs
// (precomputed per pair) into LDS, build R^0 in LDS from its closed form
// (wave_r0), and lane k, owning bra Cartesian component ab, forms
//     Y_Q = sum_{t in box(ab)} E^{ab}_t R_{t+Q}            (Q over the ket Hermite set)
//     (ab|cd) = sum_{s in box(cd)} (-1)^{|s|} E^{cd}_s Y_s  (eq. eri_formula)
// The block is accumulated over primitive quartets in LDS (or streamed in
// chunks for the largest classes) and digested into the four exchange blocks
// of the 8-fold symmetry, which are flushed to the Cartesian accumulator:
// K_ad and K_bd after every quartet, K_ac and K_bc (the same elements for all
// quartets of a work-list row) after the row's last quartet in the range.
// A workgroup walks a contiguous range of the work list, so the bra search is
// done once per range.  T is the arithmetic type of the primitive integrals
// (LDS tables and the block); the density tiles, the digestion and the
// exchange tiles are double precision.  In the mixed mode a quartet is one
// precision tile.  Most classes use the ket-first form k_wave_x below; this
// bra-first kernel serves the rest (KETFIRST in WaveCfg).
#pragma once
#include "k_pair.hpp"
#include "kern_args.hpp"
#include "md_device.hpp"
#include "wave_r.hpp"

namespace md {

template <int LA, int LB, int LC, int LD, typename T = double>
struct WaveCfg {
    static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    static constexpr int NAB = NA * NB, NCD = NC * ND, NBLK = NAB * NCD;
    static constexpr int L = LA + LB + LC + LD, LAB = LA + LB, LCD = LC + LD, L1 = L + 1;
    static constexpr int NR0 = L1 * L1 * L1;
    static constexpr bool STREAM = NBLK > 2048;
    static constexpr int NABCH = (NAB + 63) / 64;
    static constexpr int CDCH = STREAM ? 16 : NCD;
    static constexpr int NCDCH = (NCD + CDCH - 1) / CDCH;
    static constexpr int NV = STREAM ? 64 * CDCH : NBLK;
    static constexpr int SB = EprodOff<LA, LB>().off[NAB];
    // 1D Hermite tables of the bra [i][j][t] per axis (products formed on the fly)
    static constexpr int EDJ = LAB + 1, EDI = (LB + 1) * EDJ, EBD = (LA + 1) * EDI;
    static constexpr int SK = EprodOff<LC, LD>().off[NCD];
    static constexpr int ND_ = NA * NC + NA * ND + NB * NC + NB * ND;
    // quartets per range: the heaviest classes have the fewest quartets, so
    // they take short ranges to give the launch enough workgroups
    static constexpr int RANGE = L >= 11 ? 1 : (L == 10 ? 2 : 8);
    // ket-first form (k_wave_x) where it was measured faster: a lane's X
    // accumulators (bra Hermite rounds x ket components) fit in registers,
    // and the bra Hermite set (35+ indices for la + lb >= 4) fills the lanes
    static constexpr bool KETFIRST = LAB >= 4 && ((nherm(LAB) + 63) / 64) * NCD <= 72;
};

// Digest of a sub-block (streaming mode): V(ab, cd) = sV[(cd - cdb) * vstride
// + (ab - abb)] for ab in [ab0, ab1), cd in [cd0, cd1); same element-wise
// scatter with LDS atomics as digest_full.
template <int NA, int NB, int NC, int ND, typename T>
__device__ __forceinline__ void digest_rt(const T *sV, int vstride, int abb, int cdb, int ab0,
                                          int ab1, int cd0, int cd1, const double *sD, double *sK,
                                          int lane, double s)
{
    const double *D13 = sD, *D14 = sD + NA * NC, *D23 = D14 + NA * ND, *D24 = D23 + NB * NC;
    double *K13 = sK, *K14 = sK + NA * NC, *K23 = K14 + NA * ND, *K24 = K23 + NB * NC;
    const int nab = ab1 - ab0, n = nab * (cd1 - cd0);
    for (int e = lane; e < n; e += 64) {
        const int ab = ab0 + e % nab, cd = cd0 + e / nab;
        const int i = ab / NB, j = ab % NB, k = cd / ND, l = cd % ND;
        const double v = s * (double)sV[(cd - cdb) * vstride + (ab - abb)];
        atomicAdd(&K13[i * NC + k], v * D24[j * ND + l]);
        atomicAdd(&K14[i * ND + l], v * D23[j * NC + k]);
        atomicAdd(&K23[j * NC + k], v * D14[i * ND + l]);
        atomicAdd(&K24[j * ND + l], v * D13[i * NC + k]);
    }
}

// Digest of a whole block held as sV[cd * NAB + ab]: every lane takes block
// elements in turn and adds each one's four contributions
//     K_ac[i][k] += V D_bd[j][l],  K_ad[i][l] += V D_bc[j][k],
//     K_bc[j][k] += V D_ad[i][l],  K_bd[j][l] += V D_ac[i][k]
// to the LDS exchange tiles with FP64 LDS atomics (the lanes of one step share
// at most NA or NB targets, so the atomics rarely collide, and no lane waits
// on another's branch).
template <int NA, int NB, int NC, int ND, typename T>
__device__ __forceinline__ void digest_full(const T *sV, const double *sD, double *sK, int lane, double s)
{
    constexpr int NAB = NA * NB, NCD = NC * ND;
    const double *D13 = sD, *D14 = sD + NA * NC, *D23 = D14 + NA * ND, *D24 = D23 + NB * NC;
    double *K13 = sK, *K14 = sK + NA * NC, *K23 = K14 + NA * ND, *K24 = K23 + NB * NC;
    for (int e = lane; e < NAB * NCD; e += 64) {
        const int ab = e % NAB, cd = e / NAB;
        const int i = ab / NB, j = ab % NB, k = cd / ND, l = cd % ND;
        const double v = s * (double)sV[e];
        atomicAdd(&K13[i * NC + k], v * D24[j * ND + l]);
        atomicAdd(&K14[i * ND + l], v * D23[j * NC + k]);
        atomicAdd(&K23[j * NC + k], v * D14[i * ND + l]);
        atomicAdd(&K24[j * ND + l], v * D13[i * NC + k]);
    }
}

// Add the LDS exchange tiles of a quartet to the accumulator: K_ad and K_bd
// always, K_ac and K_bc (shared by the quartets of one work-list row: same
// bra, same ket shell c) only after the row's last quartet.  Each element is
// read, cleared and added by one lane; exact zeros are not added.
template <int NA, int NB, int NC, int ND>
__device__ __forceinline__ void flush_tiles(double *sK, const CPair &A, const CPair &B, double *__restrict__ Kacc,
                                            int n, bool row_end, int lane)
{
    constexpr int ND_ = NA * NC + NA * ND + NB * NC + NB * ND;
    for (int o = lane; o < ND_; o += 64) {
        int row, col;
        bool shared;
        if (o < NA * NC) { row = A.c1 + o / NC; col = B.c1 + o % NC; shared = true; }
        else if (o < NA * NC + NA * ND) { int r = o - NA * NC; row = A.c1 + r / ND; col = B.c2 + r % ND; shared = false; }
        else if (o < NA * NC + NA * ND + NB * NC) { int r = o - NA * NC - NA * ND; row = A.c2 + r / NC; col = B.c1 + r % NC; shared = true; }
        else { int r = o - NA * NC - NA * ND - NB * NC; row = A.c2 + r / ND; col = B.c2 + r % ND; shared = false; }
        if (shared && !row_end) continue;
        const double v = sK[o];
        sK[o] = 0.0;
        if (v != 0.0) unsafeAtomicAdd(&Kacc[(int64_t)row * n + col], v);
    }
}

template <int LA, int LB, int LC, int LD, typename T>
__device__ __forceinline__ void k_wave_run(const KArgs &a, int blk_x, int grid_x)
{
    using C = WaveCfg<LA, LB, LC, LD, T>;
    constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND;
    constexpr int NAB = C::NAB, NCD = C::NCD, L = C::L, L1 = C::L1, LCD = C::LCD;
    constexpr EprodOff<LC, LD> ok{};

    __shared__ T sR0[C::NR0];
    __shared__ T sF[L + 1];
    __shared__ T sH[HPolyDims<L>::N];
    __shared__ int sHerm[nherm(L)];
    __shared__ T sE1[3 * C::EBD];
    __shared__ T sEk[C::SK];
    __shared__ T sV[C::NV];
    __shared__ double sD[C::ND_];
    __shared__ double sK[C::ND_];

    const int lane = threadIdx.x;
    herm_table_lds(sHerm, nherm(L), lane);
    // per-lane R^0 term plan (L <= 9), visible after the first barrier; only
    // where the workgroup's LDS stays within 20 KB (eight workgroups per CU)
    constexpr int LDS0 = (int)sizeof(T) * (C::NR0 + L + 1 + HPolyDims<L>::N + 3 * C::EBD + C::SK + C::NV) +
                         16 * C::ND_ + 4 * nherm(L);
    constexpr bool PLAN = R0Plan<L, T>::OK && LDS0 + R0Plan<L, T>::NT * 256 <= 20480;
    __shared__ uint32_t sPlan[PLAN ? R0Plan<L, T>::NT * 64 : 1];
    R0Plan<L, T> r0p;
    r0p.code = sPlan;
    if constexpr (PLAN) r0_plan_build<L, T>(r0p, lane);
    for (int o = lane; o < C::ND_; o += 64) sK[o] = 0.0;  // cleared again by every flush

    // the bra components this lane owns: their boxes and 1D table offsets
    int own_m[C::NABCH][3], own_off[C::NABCH][3];
    bool own[C::NABCH];
#pragma unroll
    for (int r = 0; r < C::NABCH; ++r) {
        const int ab = r * 64 + lane;
        own[r] = ab < NAB;
        int ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
        if (own[r]) {
            cart_rt(LA, ab / NB, ax, ay, az);
            cart_rt(LB, ab % NB, bx, by, bz);
        }
        own_m[r][0] = ax + bx + 1;
        own_m[r][1] = ay + by + 1;
        own_m[r][2] = az + bz + 1;
        own_off[r][0] = ax * C::EDI + bx * C::EDJ;
        own_off[r][1] = C::EBD + ay * C::EDI + by * C::EDJ;
        own_off[r][2] = 2 * C::EBD + az * C::EDI + bz * C::EDJ;
    }

    const int n = a.ld;
    for (int64_t w0 = (int64_t)blk_x * C::RANGE; w0 < a.nwork; w0 += (int64_t)grid_x * C::RANGE) {
        const int64_t w1 = (w0 + C::RANGE < a.nwork) ? w0 + C::RANGE : a.nwork;
        int row = k_find_row(a.prefix, a.nrows, w0);
        int jk = (int)(w0 - a.prefix[row]);
        for (int64_t w = w0; w < w1; ++w) {
            if (w > w0) {
                ++jk;
                while (a.prefix[row] + jk >= a.prefix[row + 1]) {
                    ++row;
                    jk = 0;
                }
            }
            const int ib = a.rows[row].x, kj = a.rows[row].y + jk;
            const CPair A = a.bra[ib];
            const CPair B = a.ket[kj];
            // last quartet of its row inside this range: K_ac, K_bc are flushed after it
            const bool row_end = w + 1 == w1 || a.prefix[row] + jk + 1 >= a.prefix[row + 1];
            bool take = true;
            if (a.mode != 0 || a.tau_dens > 0.0) {  // uniform over the workgroup
                const double bound = a.Qbra[ib] * a.Qket[kj] * k_dens_bound(a.Pm, a.nsh, A, B);
                if (a.mode != 0) take = (bound >= a.tau_mix) == (a.mode == 1);
                if (bound < a.tau_dens) take = false;  // density-weighted screen
            }
            if (take) {
            double s = 1.0;
            if (A.sh1 == A.sh2) s *= 0.5;
            if (B.sh1 == B.sh2) s *= 0.5;
            if (a.same && same_pair(A, B)) s *= 0.5;

            // density blocks D_ac, D_ad, D_bc, D_bd
            for (int o = lane; o < C::ND_; o += 64) {
                int row, col;
                if (o < NA * NC) { row = A.c1 + o / NC; col = B.c1 + o % NC; }
                else if (o < NA * NC + NA * ND) { int r = o - NA * NC; row = A.c1 + r / ND; col = B.c2 + r % ND; }
                else if (o < NA * NC + NA * ND + NB * NC) { int r = o - NA * NC - NA * ND; row = A.c2 + r / NC; col = B.c1 + r % NC; }
                else { int r = o - NA * NC - NA * ND - NB * NC; row = A.c2 + r / ND; col = B.c2 + r % ND; }
                sD[o] = a.D[(int64_t)row * n + col];
            }
            if constexpr (!C::STREAM)
                for (int o = lane; o < C::NV; o += 64) sV[o] = T(0);
            __syncthreads();

            const double qk0 = a.pp[B.poff].q;
            for (int ip = 0; ip < A.np; ++ip) {
                const PrimPair pb = a.pp[A.poff + ip];
                if (pb.q * qk0 < a.tau_prim) break;
                // bra 1D tables once per bra primitive (their previous readers
                // finished at the last barrier of the previous ket loop); the
                // single-precision form folds K_ab (2p)^{t/2} in (md_device.hpp)
                if (lane < 3) {
                    const double pa = lane == 0 ? pb.PA[0] : (lane == 1 ? pb.PA[1] : pb.PA[2]);
                    const double pbb = lane == 0 ? pb.PB[0] : (lane == 1 ? pb.PB[1] : pb.PB[2]);
                    const bool f32 = sizeof(T) == 4;
                    etab_store_scaled<LA, LB, T>(pa, pbb, pb.o2p, (f32 && lane == 0) ? pb.K : 1.0,
                                                 f32 ? sqrt(2.0 * pb.p) : 1.0, sE1 + lane * C::EBD);
                }
                PairLite pk = pair_lite(a.pp + B.poff);
                for (int kp = 0; kp < B.np; ++kp) {
                    if (pb.q * pk.q < a.tau_prim) break;
                    // next ket primitive pair in flight while this one is evaluated
                    const PairLite pk_next = pair_lite(a.pp + B.poff + (kp + 1 < B.np ? kp + 1 : kp));
                    const QuartetGeo g = quartet_geo(pb, pk, a.om2);
                    wave_boys<L, T>(g, a.boys, sF, lane);
                    wave_hpoly<L, T>(g, sH, lane);
                    const T *ek = pick<T>(a.eprod_ket, a.eprodf_ket) + (int64_t)(B.poff + kp - a.pbase_ket) * C::SK;
                    for (int o = lane; o < C::SK; o += 64) sEk[o] = ek[o];
                    __syncthreads();
                    if constexpr (PLAN)
                        wave_r0h_plan<L, T>(r0p, sF, sH, sR0, lane);
                    else
                        wave_r0h<L, T>(sF, sH, sHerm, sR0, lane);
                    __syncthreads();

                    static_for<0, C::NABCH>([&](auto chc) {
                        constexpr int ch = decltype(chc)::value;
                        const int ab = ch * 64 + lane;
                        T Y[nherm(LCD)];
#pragma unroll
                        for (int q = 0; q < nherm(LCD); ++q) Y[q] = T(0);
                        if (own[ch]) {
                            // the lane's box (tx, ty, tz) walked in one flat loop whose
                            // trip count is the chunk's largest box, the same for every
                            // lane (nested per-lane loops would run the union of all
                            // lanes' boxes)
                            constexpr int BMAX = box_max(LA, LB, ch * 64, ch * 64 + 64);
                            const int mx = own_m[ch][0], my = own_m[ch][1], mz = own_m[ch][2];
                            const int nbox = mx * my * mz;
                            const T *Ex = sE1 + own_off[ch][0], *Ey = sE1 + own_off[ch][1], *Ez = sE1 + own_off[ch][2];
                            int tx = 0, ty = 0, tz = 0;
#pragma unroll 2
                            for (int st = 0; st < BMAX; ++st) {
                                if (st < nbox) {
                                    const T ev = Ex[tx] * Ey[ty] * Ez[tz];
                                    const T *Rb = sR0 + (tx * L1 + ty) * L1 + tz;
                                    static_for<0, nherm(LCD)>([&](auto qc) {
                                        constexpr int Q = decltype(qc)::value;
                                        constexpr int qo = (herm_t(Q) * L1 + herm_u(Q)) * L1 + herm_v(Q);
                                        Y[Q] += ev * Rb[qo];
                                    });
                                }
                                if (++tz == mz) {
                                    tz = 0;
                                    if (++ty == my) {
                                        ty = 0;
                                        ++tx;
                                    }
                                }
                            }
                            if constexpr (sizeof(T) == 4) {  // ket factor r^|Q| of the scaled form
                                T rp[LCD + 1];
                                powers<LCD>((T)g.r, rp);
                                static_for<0, nherm(LCD)>([&](auto qc) {
                                    constexpr int Q = decltype(qc)::value;
                                    Y[Q] *= rp[herm_t(Q) + herm_u(Q) + herm_v(Q)];
                                });
                            }
                        }
                        static_for<0, C::NCDCH>([&](auto kcc) {
                            constexpr int kc = decltype(kcc)::value;
                            constexpr int cd0 = kc * C::CDCH;
                            constexpr int cd1 = (cd0 + C::CDCH < NCD) ? cd0 + C::CDCH : NCD;
                            static_for<cd0, cd1>([&](auto cdc) {
                                constexpr int cd = decltype(cdc)::value;
                                constexpr int c = cd / ND, d = cd % ND;
                                constexpr int nsx = cart_x(LC, c) + cart_x(LD, d) + 1;
                                constexpr int nsy = cart_y(LC, c) + cart_y(LD, d) + 1;
                                constexpr int nsz = cart_z(LC, c) + cart_z(LD, d) + 1;
                                T v = T(0);
                                static_for<0, nsx * nsy * nsz>([&](auto qc) {
                                    constexpr int q = decltype(qc)::value;
                                    constexpr int sx = q / (nsy * nsz), sy = (q / nsz) % nsy, sz = q % nsz;
                                    constexpr T sg = ((sx + sy + sz) & 1) ? T(-1) : T(1);
                                    v += sg * sEk[ok.off[cd] + q] * Y[herm_idx(sx, sy, sz)];
                                });
                                if constexpr (C::STREAM) {
                                    sV[(cd - cd0) * 64 + lane] = v;
                                } else {
                                    if (ab < NAB) sV[cd * NAB + ab] += v;
                                }
                            });
                            if constexpr (C::STREAM) {
                                __syncthreads();
                                const int ab0 = ch * 64, ab1 = (ab0 + 64 < NAB) ? ab0 + 64 : NAB;
                                digest_rt<NA, NB, NC, ND, T>(sV, 64, ab0, cd0, ab0, ab1, cd0, cd1, sD, sK, lane, s);
                                __syncthreads();
                            }
                        });
                    });
                    __syncthreads();
                    pk = pk_next;
                }
            }
            if constexpr (!C::STREAM) {
                digest_full<NA, NB, NC, ND, T>(sV, sD, sK, lane, s);
                __syncthreads();
            }
            }  // take
            flush_tiles<NA, NB, NC, ND>(sK, A, B, a.Kacc, n, row_end, lane);
            __syncthreads();
        }
    }
}

template <int LA, int LB, int LC, int LD, typename T>
__global__ __launch_bounds__(64) void k_wave(KArgs a)
{
    k_wave_run<LA, LB, LC, LD, T>(a, blockIdx.x, gridDim.x);
}

// batch form: workgroup b runs block (items[b].y, items[b].z) of the
// launch whose arguments are tab[items[b].x]
template <int LA, int LB, int LC, int LD, typename T>
__global__ __launch_bounds__(64) void k_wave_q(const KArgs *__restrict__ tab, const int4 *__restrict__ items)
{
    const int4 it = items[blockIdx.x];
    KArgs a = tab[it.x];
    globalize(a);
    k_wave_run<LA, LB, LC, LD, T>(a, it.y, it.w);
}

// Ket-first form for the classes whose block fits in LDS.  Per primitive
// quartet, for each ket component cd (a compile-time round in which every
// lane takes the same path), lane k owning the bra Hermite index t forms
//     X_t(cd) += sum_{s in box(cd)} (-1)^{|s|} E^{cd}_s R_{t+s}
// and keeps the sum in registers over the ket primitive pairs.  After the
// ket primitives of one bra primitive pair, the lanes owning bra components
// ab apply the bra transform once:
//     V(ab, cd) += sum_{t in box(ab)} E^{ab}_t X_t(cd)
// (eq. eri_formula with the two Hermite sums in the other order), so the
// bra transform runs per bra primitive pair instead of per primitive quartet.
// The lane then digests its block row at once (digestion is linear in the
// block), so no block buffer is needed and large blocks fit too.
template <int LA, int LB, int LC, int LD, typename T>
__device__ __forceinline__ void k_wave_x_run(const KArgs &a, int blk_x, int grid_x)
{
    using C = WaveCfg<LA, LB, LC, LD, T>;
    constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND;
    constexpr int NAB = C::NAB, NCD = C::NCD, L = C::L, L1 = C::L1, LAB = C::LAB, LCD = C::LCD;
    constexpr int NHAB = nherm(LAB), TCH = (NHAB + 63) / 64;
    constexpr EprodOff<LC, LD> ok{};
    static_assert(C::KETFIRST, "ket-first form: X of a lane fits in registers");

    // R^0 lives during the ket loop, X only between its end and the bra
    // transform (separated by barriers), so they share one buffer
    // R^0 at t ST + u SU + v; the t stride is padded by two off the power of
    // two so that lanes whose indices differ only in t hit different LDS banks
    constexpr int SU = L1, ST = L1 * L1 + 2, NR0P = L1 * ST;
    constexpr int NRX = NR0P > NCD * NHAB ? NR0P : NCD * NHAB;
    __shared__ T sRX[NRX];
    T *const sR0 = sRX;
    T *const sX = sRX;
    // geometry and scaled Boys values of a batch of ket primitive pairs
    constexpr int NBAT = 64 / (L + 1);
    __shared__ T sFb[NBAT * (L + 1)];
    __shared__ double sGeo[NBAT * 6];
    __shared__ T sH[HPolyDims<L>::N];
    __shared__ int sHerm[nherm(L)];
    __shared__ T sE1[3 * C::EBD];
    __shared__ T sEk[C::SK];
    __shared__ double sD[C::ND_];
    __shared__ double sK[C::ND_];

    const int lane = threadIdx.x;
    herm_table_lds(sHerm, nherm(L), lane);
    // per-lane R^0 term plan (the classes with L <= 9), visible after the
    // first barrier of the quartet loop; only where the workgroup's LDS stays
    // within 20 KB (eight workgroups per CU)
    constexpr int LDS0 = (int)sizeof(T) * (NRX + NBAT * (L + 1) + HPolyDims<L>::N + 3 * C::EBD + C::SK) +
                         8 * (NBAT * 6 + 2 * C::ND_) + 4 * nherm(L);
    constexpr bool PLAN = R0Plan<L, T>::OK && LDS0 + R0Plan<L, T>::NT * 256 <= 20480;
    __shared__ uint32_t sPlan[PLAN ? R0Plan<L, T>::NT * 64 : 1];
    R0Plan<L, T> r0p;
    r0p.code = sPlan;
    if constexpr (PLAN) r0_plan_build<L, T, ST, SU>(r0p, lane);
    for (int o = lane; o < C::ND_; o += 64) sK[o] = 0.0;  // cleared again by every flush

    // bra Hermite indices this lane owns in the ket rounds
    int tof[TCH];
    bool town[TCH];
#pragma unroll
    for (int r = 0; r < TCH; ++r) {
        const int t = r * 64 + lane;
        town[r] = t < NHAB;
        const int code = c_herm.tuv[town[r] ? t : 0];
        tof[r] = (code & 0xff) * ST + ((code >> 8) & 0xff) * SU + (code >> 16);
    }
    // bra components this lane owns in the bra transform
    int own_m[C::NABCH][3], own_off[C::NABCH][3];
    bool own[C::NABCH];
#pragma unroll
    for (int r = 0; r < C::NABCH; ++r) {
        const int ab = r * 64 + lane;
        own[r] = ab < NAB;
        int ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
        if (own[r]) {
            cart_rt(LA, ab / NB, ax, ay, az);
            cart_rt(LB, ab % NB, bx, by, bz);
        }
        own_m[r][0] = ax + bx + 1;
        own_m[r][1] = ay + by + 1;
        own_m[r][2] = az + bz + 1;
        own_off[r][0] = ax * C::EDI + bx * C::EDJ;
        own_off[r][1] = C::EBD + ay * C::EDI + by * C::EDJ;
        own_off[r][2] = 2 * C::EBD + az * C::EDI + bz * C::EDJ;
    }

    const int n = a.ld;
    for (int64_t w0 = (int64_t)blk_x * C::RANGE; w0 < a.nwork; w0 += (int64_t)grid_x * C::RANGE) {
        const int64_t w1 = (w0 + C::RANGE < a.nwork) ? w0 + C::RANGE : a.nwork;
        int row = k_find_row(a.prefix, a.nrows, w0);
        int jk = (int)(w0 - a.prefix[row]);
        for (int64_t w = w0; w < w1; ++w) {
            if (w > w0) {
                ++jk;
                while (a.prefix[row] + jk >= a.prefix[row + 1]) {
                    ++row;
                    jk = 0;
                }
            }
            const int ib = a.rows[row].x, kj = a.rows[row].y + jk;
            const CPair A = a.bra[ib];
            const CPair B = a.ket[kj];
            // last quartet of its row inside this range: K_ac, K_bc are flushed after it
            const bool row_end = w + 1 == w1 || a.prefix[row] + jk + 1 >= a.prefix[row + 1];
            bool take = true;
            if (a.mode != 0 || a.tau_dens > 0.0) {  // uniform over the workgroup
                const double bound = a.Qbra[ib] * a.Qket[kj] * k_dens_bound(a.Pm, a.nsh, A, B);
                if (a.mode != 0) take = (bound >= a.tau_mix) == (a.mode == 1);
                if (bound < a.tau_dens) take = false;  // density-weighted screen
            }
            if (take) {
            double s = 1.0;
            if (A.sh1 == A.sh2) s *= 0.5;
            if (B.sh1 == B.sh2) s *= 0.5;
            if (a.same && same_pair(A, B)) s *= 0.5;

            for (int o = lane; o < C::ND_; o += 64) {
                int row, col;
                if (o < NA * NC) { row = A.c1 + o / NC; col = B.c1 + o % NC; }
                else if (o < NA * NC + NA * ND) { int r = o - NA * NC; row = A.c1 + r / ND; col = B.c2 + r % ND; }
                else if (o < NA * NC + NA * ND + NB * NC) { int r = o - NA * NC - NA * ND; row = A.c2 + r / NC; col = B.c1 + r % NC; }
                else { int r = o - NA * NC - NA * ND - NB * NC; row = A.c2 + r / ND; col = B.c2 + r % ND; }
                sD[o] = a.D[(int64_t)row * n + col];
            }
            __syncthreads();

            const double qk0 = a.pp[B.poff].q;
            for (int ip = 0; ip < A.np; ++ip) {
                const PrimPair pb = a.pp[A.poff + ip];
                if (pb.q * qk0 < a.tau_prim) break;
                // bra 1D tables of this bra primitive pair (read again only by
                // the bra transform below, after the ket loop's last barrier)
                if (lane < 3) {
                    const double pa = lane == 0 ? pb.PA[0] : (lane == 1 ? pb.PA[1] : pb.PA[2]);
                    const double pbb = lane == 0 ? pb.PB[0] : (lane == 1 ? pb.PB[1] : pb.PB[2]);
                    const bool f32 = sizeof(T) == 4;
                    etab_store_scaled<LA, LB, T>(pa, pbb, pb.o2p, (f32 && lane == 0) ? pb.K : 1.0,
                                                 f32 ? sqrt(2.0 * pb.p) : 1.0, sE1 + lane * C::EBD);
                }
                T X[TCH][NCD];
#pragma unroll
                for (int r = 0; r < TCH; ++r)
#pragma unroll
                    for (int cd = 0; cd < NCD; ++cd) X[r][cd] = T(0);

                bool screened = false;
                for (int kb = 0; kb < B.np && !screened; kb += NBAT) {
                    // one pass for a batch of ket primitive pairs: lane o owns
                    // (kp, m) = (kb + o / (L + 1), o % (L + 1)) and forms
                    // pref (-2 alpha)^m F_m (scaled form: pref0 w^m F_m); the
                    // m = 0 lane also keeps the pair's geometry
                    {
                        const int kq = kb + lane / (L + 1), m = lane % (L + 1);
                        if (lane < NBAT * (L + 1) && kq < B.np) {
                            const PairLite pq = pair_lite(a.pp + B.poff + kq);
                            const QuartetGeo gq = quartet_geo(pb, pq, a.om2);
                            const double F = boys_one(m, gq.T, a.boys);
                            const double sc = sizeof(T) == 4 ? gq.pref0 : gq.pref;
                            const double m2a = sizeof(T) == 4 ? gq.w : -2.0 * gq.alpha;
                            sFb[(kq - kb) * (L + 1) + m] = (T)(sc * pow_small<L>(m2a, m) * F);
                            if (m == 0) {
                                double *o = sGeo + (kq - kb) * 6;
                                o[0] = gq.X;
                                o[1] = gq.Y;
                                o[2] = gq.Z;
                                o[3] = gq.c;
                                o[4] = gq.r;
                                o[5] = pq.q;
                            }
                        }
                    }
                    __syncthreads();
                    const int ke = (kb + NBAT < B.np) ? kb + NBAT : B.np;
                    for (int kp = kb; kp < ke; ++kp) {
                        const double *gk = sGeo + (kp - kb) * 6;
                        if (pb.q * gk[5] < a.tau_prim) {  // uniform: the pairs are sorted by q
                            screened = true;
                            break;
                        }
                        QuartetGeo g;
                        g.X = gk[0];
                        g.Y = gk[1];
                        g.Z = gk[2];
                        g.c = gk[3];
                        g.r = gk[4];
                        wave_hpoly<L, T>(g, sH, lane);
                        const T *ek = pick<T>(a.eprod_ket, a.eprodf_ket) + (int64_t)(B.poff + kp - a.pbase_ket) * C::SK;
                        for (int o = lane; o < C::SK; o += 64) sEk[o] = ek[o];
                        __syncthreads();
                        if constexpr (PLAN)
                            wave_r0h_plan<L, T, ST, SU>(r0p, sFb + (kp - kb) * (L + 1), sH, sR0, lane);
                        else
                            wave_r0h<L, T, ST, SU>(sFb + (kp - kb) * (L + 1), sH, sHerm, sR0, lane);
                        __syncthreads();

                        T rp[LCD + 1];  // r^|s| of the scaled single-precision form
                        if constexpr (sizeof(T) == 4) powers<LCD>((T)g.r, rp);
                        static_for<0, NCD>([&](auto cdc) {
                            constexpr int cd = decltype(cdc)::value;
                            constexpr int c = cd / ND, d = cd % ND;
                            constexpr int nsx = cart_x(LC, c) + cart_x(LD, d) + 1;
                            constexpr int nsy = cart_y(LC, c) + cart_y(LD, d) + 1;
                            constexpr int nsz = cart_z(LC, c) + cart_z(LD, d) + 1;
                            T e[nsx * nsy * nsz];
                            static_for<0, nsx * nsy * nsz>([&](auto qc) {
                                constexpr int q = decltype(qc)::value;
                                constexpr int sx = q / (nsy * nsz), sy = (q / nsz) % nsy, sz = q % nsz;
                                constexpr T sg = ((sx + sy + sz) & 1) ? T(-1) : T(1);
                                if constexpr (sizeof(T) == 4)
                                    e[q] = sg * rp[sx + sy + sz] * sEk[ok.off[cd] + q];
                                else
                                    e[q] = sg * sEk[ok.off[cd] + q];
                            });
    #pragma unroll
                            for (int r = 0; r < TCH; ++r) {
                                if (!town[r]) continue;
                                const T *Rb = sR0 + tof[r];
                                T x = T(0);
                                static_for<0, nsx * nsy * nsz>([&](auto qc) {
                                    constexpr int q = decltype(qc)::value;
                                    constexpr int sx = q / (nsy * nsz), sy = (q / nsz) % nsy, sz = q % nsz;
                                    x += e[q] * Rb[sx * ST + sy * SU + sz];
                                });
                                X[r][cd] += x;
                            }
                        });
                        __syncthreads();
                    }
                }

                // bra transform of this bra primitive pair
#pragma unroll
                for (int r = 0; r < TCH; ++r)
                    if (town[r])
#pragma unroll
                        for (int cd = 0; cd < NCD; ++cd) sX[cd * NHAB + r * 64 + lane] = X[r][cd];
                __syncthreads();
                static_for<0, C::NABCH>([&](auto chc) {
                    constexpr int ch = decltype(chc)::value;
                    const int ab = ch * 64 + lane;
                    if (own[ch]) {
                        constexpr int BMAX = box_max(LA, LB, ch * 64, ch * 64 + 64);
                        const int mx = own_m[ch][0], my = own_m[ch][1], mz = own_m[ch][2];
                        const int nbox = mx * my * mz;
                        const T *Ex = sE1 + own_off[ch][0], *Ey = sE1 + own_off[ch][1], *Ez = sE1 + own_off[ch][2];
                        T v[NCD];
#pragma unroll
                        for (int cd = 0; cd < NCD; ++cd) v[cd] = T(0);
                        int tx = 0, ty = 0, tz = 0;
                        for (int st = 0; st < BMAX; ++st) {
                            if (st < nbox) {
                                const T ev = Ex[tx] * Ey[ty] * Ez[tz];
                                const T *xr = sX + herm_idx_rt(tx, ty, tz);
#pragma unroll
                                for (int cd = 0; cd < NCD; ++cd) v[cd] += ev * xr[cd * NHAB];
                            }
                            if (++tz == mz) {
                                tz = 0;
                                if (++ty == my) {
                                    ty = 0;
                                    ++tx;
                                }
                            }
                        }
                        // digest this bra primitive pair's block row ab directly
                        // (digestion is linear in the block): per exchange element
                        // one LDS atomic with the row's sum over the other index
                        const int i = ab / NB, j = ab % NB;
                        const double *D13 = sD, *D14 = sD + NA * NC, *D23 = D14 + NA * ND, *D24 = D23 + NB * NC;
                        double *K13 = sK, *K14 = sK + NA * NC, *K23 = K14 + NA * ND, *K24 = K23 + NB * NC;
                        double d13[NC], d23[NC], d14[ND], d24[ND];
#pragma unroll
                        for (int k = 0; k < NC; ++k) {
                            d13[k] = D13[i * NC + k];
                            d23[k] = D23[j * NC + k];
                        }
#pragma unroll
                        for (int l = 0; l < ND; ++l) {
                            d14[l] = D14[i * ND + l];
                            d24[l] = D24[j * ND + l];
                        }
#pragma unroll
                        for (int k = 0; k < NC; ++k) {
                            double t13 = 0.0, t23 = 0.0;
#pragma unroll
                            for (int l = 0; l < ND; ++l) {
                                t13 += (double)v[k * ND + l] * d24[l];
                                t23 += (double)v[k * ND + l] * d14[l];
                            }
                            atomicAdd(&K13[i * NC + k], s * t13);
                            atomicAdd(&K23[j * NC + k], s * t23);
                        }
#pragma unroll
                        for (int l = 0; l < ND; ++l) {
                            double t14 = 0.0, t24 = 0.0;
#pragma unroll
                            for (int k = 0; k < NC; ++k) {
                                t14 += (double)v[k * ND + l] * d23[k];
                                t24 += (double)v[k * ND + l] * d13[k];
                            }
                            atomicAdd(&K14[i * ND + l], s * t14);
                            atomicAdd(&K24[j * ND + l], s * t24);
                        }
                    }
                });
                __syncthreads();
            }
            }  // take
            flush_tiles<NA, NB, NC, ND>(sK, A, B, a.Kacc, n, row_end, lane);
            __syncthreads();
        }
    }
}

template <int LA, int LB, int LC, int LD, typename T>
__global__ __launch_bounds__(64) void k_wave_x(KArgs a)
{
    k_wave_x_run<LA, LB, LC, LD, T>(a, blockIdx.x, gridDim.x);
}

// batch form: workgroup b runs block (items[b].y, items[b].z) of the
// launch whose arguments are tab[items[b].x]
template <int LA, int LB, int LC, int LD, typename T>
__global__ __launch_bounds__(64) void k_wave_x_q(const KArgs *__restrict__ tab, const int4 *__restrict__ items)
{
    const int4 it = items[blockIdx.x];
    KArgs a = tab[it.x];
    globalize(a);
    k_wave_x_run<LA, LB, LC, LD, T>(a, it.y, it.w);
}

template <int LA, int LB, int LC, int LD>
void launch_k_wave_t(const KArgs &a, bool fp32, hipStream_t st)
{
    using C = WaveCfg<LA, LB, LC, LD>;
    const int64_t ranges = (a.nwork + C::RANGE - 1) / C::RANGE;
    const int64_t cap = a.grid_cap > 0 ? a.grid_cap : 32768;
    const int64_t blocks = ranges < cap ? ranges : cap;
    if (blocks <= 0) return;
    if (queue_sink()) {  // a batch plan: each block walks ranges/blocks ranges
        QueueLaunchFn fn;
        if constexpr (C::KETFIRST)
            fn = fp32 ? &queue_launch<KArgs, k_wave_x_q<LA, LB, LC, LD, float>, 64>
                      : &queue_launch<KArgs, k_wave_x_q<LA, LB, LC, LD, double>, 64>;
        else
            fn = fp32 ? &queue_launch<KArgs, k_wave_q<LA, LB, LC, LD, float>, 64>
                      : &queue_launch<KArgs, k_wave_q<LA, LB, LC, LD, double>, 64>;
        queue_record(fn, a, (int)blocks, 1,
                     (double)ranges / (double)blocks, C::KETFIRST ? "k_wave_x" : "k_wave");
        return;
    }
    if constexpr (!C::KETFIRST) {
        if (fp32)
            hipLaunchKernelGGL((k_wave<LA, LB, LC, LD, float>), dim3((unsigned)blocks), dim3(64), 0, st, a);
        else
            hipLaunchKernelGGL((k_wave<LA, LB, LC, LD, double>), dim3((unsigned)blocks), dim3(64), 0, st, a);
    } else {
        if (fp32)
            hipLaunchKernelGGL((k_wave_x<LA, LB, LC, LD, float>), dim3((unsigned)blocks), dim3(64), 0, st, a);
        else
            hipLaunchKernelGGL((k_wave_x<LA, LB, LC, LD, double>), dim3((unsigned)blocks), dim3(64), 0, st, a);
    }
}

}  // namespace md
