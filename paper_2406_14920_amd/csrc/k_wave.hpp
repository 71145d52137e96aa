// k_wave.hip -- exchange (K) for angular classes whose Cartesian block is too
// large for one lane: one 64-lane workgroup evaluates one canonical contracted
// shell quartet at a time.  Per primitive quartet the wave builds R^0 in LDS
// (eq. R_recursion); lane k owns bra Cartesian component ab and forms
//     Y_Q = sum_{t in box(ab)} E^{ab}_t R_{t+Q}            (Q over the ket Hermite set)
//     (ab|cd) = sum_{s in box(cd)} (-1)^{|s|} E^{cd}_s Y_s  (eq. eri_formula)
// The block is accumulated over primitive quartets in LDS (or streamed in
// chunks for the largest classes) and digested into the four exchange blocks
// of the 8-fold symmetry, which are flushed to the Cartesian accumulator.
#pragma once
#include "kern_args.hpp"
#include "md_device.hpp"
#include "wave_r.hpp"

namespace md {

template <int LC, int LD>
struct KetBoxes {
    static constexpr int NCD = ncart(LC) * ncart(LD);
    int off[NCD + 1];
    constexpr KetBoxes() : off()
    {
        int o = 0;
        for (int cd = 0; cd < NCD; ++cd) {
            off[cd] = o;
            o += box_nnz(LC, cd / ncart(LD), LD, cd % ncart(LD));
        }
        off[NCD] = o;
    }
};

template <int LA, int LB, int LC, int LD>
struct WaveCfg {
    static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    static constexpr int NAB = NA * NB, NCD = NC * ND, NBLK = NAB * NCD;
    static constexpr int L = LA + LB + LC + LD, LAB = LA + LB, LCD = LC + LD, L1 = L + 1;
    static constexpr int NR0 = L1 * L1 * L1;
    static constexpr int NLEV = nherm(L > 0 ? L - 1 : 0);
    static constexpr bool STREAM = NBLK > 2048;
    static constexpr int NABCH = (NAB + 63) / 64;
    static constexpr int CDCH = STREAM ? 16 : NCD;
    static constexpr int NCDCH = (NCD + CDCH - 1) / CDCH;
    static constexpr int NV = STREAM ? 64 * CDCH : NBLK;
    static constexpr int EB = 3 * (LA + 1) * (LB + 1) * (LAB + 1);
    static constexpr int EK = 3 * (LC + 1) * (LD + 1) * (LCD + 1);
    static constexpr int NKP = KetBoxes<LC, LD>().off[NCD];
    static constexpr int ND_ = NA * NC + NA * ND + NB * NC + NB * ND;
};

// Digest the sub-block ab in [ab0,ab1), cd in [cd0,cd1) held in sV into the
// four exchange tiles.  vstride: ab stride of sV (NAB in accumulate mode, 64
// when streaming); sV(ab,cd) = sV[(cd - cdb) * vstride + (ab - abb)].
template <int NA, int NB, int NC, int ND>
__device__ __forceinline__ void digest(const double *sV, int vstride, int abb, int cdb, int ab0,
                                       int ab1, int cd0, int cd1, const double *sD, double *sK,
                                       int lane)
{
    const double *D13 = sD, *D14 = sD + NA * NC, *D23 = D14 + NA * ND, *D24 = D23 + NB * NC;
    double *K13 = sK, *K14 = sK + NA * NC, *K23 = K14 + NA * ND, *K24 = K23 + NB * NC;
    constexpr int O1 = NA * NC, O2 = O1 + NA * ND, O3 = O2 + NB * NC, O4 = O3 + NB * ND;
    auto V = [&](int ab, int cd) { return sV[(cd - cdb) * vstride + (ab - abb)]; };
    for (int o = lane; o < O4; o += 64) {
        double acc = 0.0;
        if (o < O1) {  // K_ac[i][k] += sum_{j,l} V[ij][kl] D_bd[j][l]
            const int i = o / NC, k = o % NC;
            const int j0 = max(0, ab0 - i * NB), j1 = min(NB, ab1 - i * NB);
            const int l0 = max(0, cd0 - k * ND), l1 = min(ND, cd1 - k * ND);
            for (int j = j0; j < j1; ++j)
                for (int l = l0; l < l1; ++l) acc += V(i * NB + j, k * ND + l) * D24[j * ND + l];
            K13[o] += acc;
        } else if (o < O2) {  // K_ad[i][l] += sum_{j,k} V[ij][kl] D_bc[j][k]
            const int r = o - O1, i = r / ND, l = r % ND;
            const int j0 = max(0, ab0 - i * NB), j1 = min(NB, ab1 - i * NB);
            for (int j = j0; j < j1; ++j)
                for (int k = 0; k < NC; ++k) {
                    const int cd = k * ND + l;
                    if (cd >= cd0 && cd < cd1) acc += V(i * NB + j, cd) * D23[j * NC + k];
                }
            K14[r] += acc;
        } else if (o < O3) {  // K_bc[j][k] += sum_{i,l} V[ij][kl] D_ad[i][l]
            const int r = o - O2, j = r / NC, k = r % NC;
            const int l0 = max(0, cd0 - k * ND), l1 = min(ND, cd1 - k * ND);
            for (int i = 0; i < NA; ++i) {
                const int ab = i * NB + j;
                if (ab < ab0 || ab >= ab1) continue;
                for (int l = l0; l < l1; ++l) acc += V(ab, k * ND + l) * D14[i * ND + l];
            }
            K23[r] += acc;
        } else {  // K_bd[j][l] += sum_{i,k} V[ij][kl] D_ac[i][k]
            const int r = o - O3, j = r / ND, l = r % ND;
            for (int i = 0; i < NA; ++i) {
                const int ab = i * NB + j;
                if (ab < ab0 || ab >= ab1) continue;
                for (int k = 0; k < NC; ++k) {
                    const int cd = k * ND + l;
                    if (cd >= cd0 && cd < cd1) acc += V(ab, cd) * D13[i * NC + k];
                }
            }
            K24[r] += acc;
        }
    }
}

template <int LA, int LB, int LC, int LD>
__global__ __launch_bounds__(64) void k_wave(KArgs a)
{
    using C = WaveCfg<LA, LB, LC, LD>;
    constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND;
    constexpr int NAB = C::NAB, NCD = C::NCD, L = C::L, L1 = C::L1, LAB = C::LAB, LCD = C::LCD;
    constexpr KetBoxes<LC, LD> kb{};

    __shared__ double sR0[C::NR0];
    __shared__ double sF[L + 1];
    __shared__ double sPow[3 * (L + 1)];
    __shared__ double sEb[C::EB];
    __shared__ double sEk[C::EK];
    __shared__ double sEkp[C::NKP];
    __shared__ double sV[C::NV];
    __shared__ double sD[C::ND_];
    __shared__ double sK[C::ND_];

    const int lane = threadIdx.x;
    constexpr int EBD = (LA + 1) * (LB + 1) * (LAB + 1);
    constexpr int EKD = (LC + 1) * (LD + 1) * (LCD + 1);

    for (int64_t w = blockIdx.x; w < a.nwork; w += gridDim.x) {
        int lo = 0, hi = a.nbra;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (a.prefix[mid] <= w) lo = mid; else hi = mid;
        }
        const int ib = lo;
        const int jk = (int)(w - a.prefix[ib]);
        const CPair A = a.bra[ib];
        const CPair B = a.ket[jk];
        const int n = a.ld;

        // density blocks D_ac, D_ad, D_bc, D_bd and zeroed exchange tiles
        for (int o = lane; o < C::ND_; o += 64) {
            int row, col;
            if (o < NA * NC) { row = A.c1 + o / NC; col = B.c1 + o % NC; }
            else if (o < NA * NC + NA * ND) { int r = o - NA * NC; row = A.c1 + r / ND; col = B.c2 + r % ND; }
            else if (o < NA * NC + NA * ND + NB * NC) { int r = o - NA * NC - NA * ND; row = A.c2 + r / NC; col = B.c1 + r % NC; }
            else { int r = o - NA * NC - NA * ND - NB * NC; row = A.c2 + r / ND; col = B.c2 + r % ND; }
            sD[o] = a.D[(int64_t)row * n + col];
            sK[o] = 0.0;
        }
        if constexpr (!C::STREAM)
            for (int o = lane; o < C::NV; o += 64) sV[o] = 0.0;
        __syncthreads();

        const double qk0 = a.pp[B.poff].q;
        for (int ip = 0; ip < A.np; ++ip) {
            const PrimPair pb = a.pp[A.poff + ip];
            if (pb.q * qk0 < a.tau_prim) break;
            for (int kp = 0; kp < B.np; ++kp) {
                const PrimPair pk = a.pp[B.poff + kp];
                if (pb.q * pk.q < a.tau_prim) break;
                const QuartetGeo g = quartet_geo(pb, pk);
                wave_boys<L>(g, a.boys, sF, lane);
                wave_powers<L>(g, sPow, lane);
                if (lane >= 61) {  // 1D Hermite tables, bra on 61..63
                    const int ax = lane - 61;
                    const double pa = ax == 0 ? pb.PA[0] : (ax == 1 ? pb.PA[1] : pb.PA[2]);
                    const double pbb = ax == 0 ? pb.PB[0] : (ax == 1 ? pb.PB[1] : pb.PB[2]);
                    etab_reg_store<LA, LB>(pa, pbb, pb.o2p, sEb + ax * EBD);
                } else if (lane >= 58) {  // ket on 58..60
                    const int ax = lane - 58;
                    const double pa = ax == 0 ? pk.PA[0] : (ax == 1 ? pk.PA[1] : pk.PA[2]);
                    const double pbb = ax == 0 ? pk.PB[0] : (ax == 1 ? pk.PB[1] : pk.PB[2]);
                    etab_reg_store<LC, LD>(pa, pbb, pk.o2p, sEk + ax * EKD);
                }
                __syncthreads();
                // ket products (-1)^{|s|} E^{cd}_s, layout per cd box [sx][sy][sz]
                for (int cd = lane; cd < NCD; cd += 64) {
                    int cx, cy, cz, dx, dy, dz;
                    cart_rt(LC, cd / ND, cx, cy, cz);
                    cart_rt(LD, cd % ND, dx, dy, dz);
                    const int ny = cy + dy + 1, nz = cz + dz + 1;
                    const double *Ex = sEk + (cx * (LD + 1) + dx) * (LCD + 1);
                    const double *Ey = sEk + EKD + (cy * (LD + 1) + dy) * (LCD + 1);
                    const double *Ez = sEk + 2 * EKD + (cz * (LD + 1) + dz) * (LCD + 1);
                    int koff = 0;
                    for (int e = 0; e < cd; ++e) {
                        int ex_, ey_, ez_, fx_, fy_, fz_;
                        cart_rt(LC, e / ND, ex_, ey_, ez_);
                        cart_rt(LD, e % ND, fx_, fy_, fz_);
                        koff += (ex_ + fx_ + 1) * (ey_ + fy_ + 1) * (ez_ + fz_ + 1);
                    }
                    double *out = sEkp + koff;
                    for (int sx = 0; sx <= cx + dx; ++sx)
                        for (int sy = 0; sy < ny; ++sy)
                            for (int sz = 0; sz < nz; ++sz) {
                                const double sg = ((sx + sy + sz) & 1) ? -1.0 : 1.0;
                                out[(sx * ny + sy) * nz + sz] = sg * Ex[sx] * Ey[sy] * Ez[sz];
                            }
                }
                wave_r0<L>(sF, sPow, sR0, lane);
                __syncthreads();

                // contraction: lane owns bra component ab = ch*64 + lane
                static_for<0, C::NABCH>([&](auto chc) {
                    constexpr int ch = decltype(chc)::value;
                    const int ab = ch * 64 + lane;
                    double Y[nherm(LCD)];
#pragma unroll
                    for (int q = 0; q < nherm(LCD); ++q) Y[q] = 0.0;
                    if (ab < NAB) {
                        int ax, ay, az, bx, by, bz;
                        cart_rt(LA, ab / NB, ax, ay, az);
                        cart_rt(LB, ab % NB, bx, by, bz);
                        const double *Ex = sEb + (ax * (LB + 1) + bx) * (LAB + 1);
                        const double *Ey = sEb + EBD + (ay * (LB + 1) + by) * (LAB + 1);
                        const double *Ez = sEb + 2 * EBD + (az * (LB + 1) + bz) * (LAB + 1);
                        for (int tx = 0; tx <= ax + bx; ++tx) {
                            const double ex = Ex[tx];
                            for (int ty = 0; ty <= ay + by; ++ty) {
                                const double exy = ex * Ey[ty];
                                for (int tz = 0; tz <= az + bz; ++tz) {
                                    const double e = exy * Ez[tz];
                                    const double *Rb = sR0 + (tx * L1 + ty) * L1 + tz;
                                    static_for<0, nherm(LCD)>([&](auto qc) {
                                        constexpr int Q = decltype(qc)::value;
                                        constexpr int qo = (herm_t(Q) * L1 + herm_u(Q)) * L1 + herm_v(Q);
                                        Y[Q] += e * Rb[qo];
                                    });
                                }
                            }
                        }
                    }
                    // (ab|cd) for every cd, or chunk by chunk when streaming
                    static_for<0, C::NCDCH>([&](auto kcc) {
                        constexpr int kc = decltype(kcc)::value;
                        constexpr int cd0 = kc * C::CDCH;
                        constexpr int cd1 = (cd0 + C::CDCH < NCD) ? cd0 + C::CDCH : NCD;
                        static_for<cd0, cd1>([&](auto cdc) {
                            constexpr int cd = decltype(cdc)::value;
                            constexpr int c = cd / ND, d = cd % ND;
                            constexpr int nsy = cart_y(LC, c) + cart_y(LD, d) + 1;
                            constexpr int nsz = cart_z(LC, c) + cart_z(LD, d) + 1;
                            constexpr int nsx = cart_x(LC, c) + cart_x(LD, d) + 1;
                            const double *ek = sEkp + kb.off[cd];
                            double v = 0.0;
                            static_for<0, nsx>([&](auto sxc) {
                                constexpr int sx = decltype(sxc)::value;
                                static_for<0, nsy>([&](auto syc) {
                                    constexpr int sy = decltype(syc)::value;
                                    static_for<0, nsz>([&](auto szc) {
                                        constexpr int sz = decltype(szc)::value;
                                        v += ek[(sx * nsy + sy) * nsz + sz] * Y[herm_idx(sx, sy, sz)];
                                    });
                                });
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
                            digest<NA, NB, NC, ND>(sV, 64, ab0, cd0, ab0, ab1, cd0, cd1, sD, sK, lane);
                            __syncthreads();
                        }
                    });
                });
                __syncthreads();
            }
        }
        if constexpr (!C::STREAM) {
            digest<NA, NB, NC, ND>(sV, NAB, 0, 0, 0, NAB, 0, NCD, sD, sK, lane);
            __syncthreads();
        }
        double s = 1.0;
        if (A.sh1 == A.sh2) s *= 0.5;
        if (B.sh1 == B.sh2) s *= 0.5;
        if (a.same && ib == jk) s *= 0.5;
        for (int o = lane; o < C::ND_; o += 64) {
            int row, col;
            if (o < NA * NC) { row = A.c1 + o / NC; col = B.c1 + o % NC; }
            else if (o < NA * NC + NA * ND) { int r = o - NA * NC; row = A.c1 + r / ND; col = B.c2 + r % ND; }
            else if (o < NA * NC + NA * ND + NB * NC) { int r = o - NA * NC - NA * ND; row = A.c2 + r / NC; col = B.c1 + r % NC; }
            else { int r = o - NA * NC - NA * ND - NB * NC; row = A.c2 + r / ND; col = B.c2 + r % ND; }
            unsafeAtomicAdd(&a.Kacc[(int64_t)row * n + col], s * sK[o]);
        }
        __syncthreads();
    }
}


template <int LA, int LB, int LC, int LD>
void launch_k_wave_t(const KArgs &a, hipStream_t st)
{
    int64_t blocks = a.nwork < 16384 ? a.nwork : 16384;
    if (blocks <= 0) return;
    hipLaunchKernelGGL((k_wave<LA, LB, LC, LD>), dim3((unsigned)blocks), dim3(64), 0, st, a);
}

}  // namespace md
