// k_pair.hpp -- exchange (K) with the bra shared by a wavefront: one
// workgroup (64 lanes) takes one bra contracted pair (ab| and up to 64
// consecutive kets |cd) of its work list, one ket per lane.  The bra's Hermite products
// E^{ab}_t come precomputed from HBM through wave-uniform loads, so the
// registers hold only what differs per lane: the auxiliary integrals R^0 of
// the lane's primitive quartet (eq. R_recursion), the ket Hermite products,
// and a chunk of the contracted Cartesian block
//     (ab|cd) = sum_t E^{ab}_t sum_s (-1)^{|s|} E^{cd}_s R_{t+s}    (eq. eri_formula)
// accumulated over the primitive quartets.  Blocks larger than the register
// budget are produced in compile-time passes over (ab, cd) chunks, R being
// rebuilt per pass.  Each finished chunk is digested by the lane into the
// four exchange blocks of the 8-fold symmetry and added to the accumulator;
// the K_ac and K_bc terms of lanes in one work-list row (same ket shell c;
// K_ad and K_bd when the kets are grouped by d) are summed across those lanes
// first.  A density-weighted screen may skip lanes.
// T is the arithmetic type of the primitive integrals (the digestion is in
// double precision); in the mixed mode a workgroup is one precision tile.
#pragma once
#include "kern_args.hpp"
#include "md_device.hpp"
#include "queue.hpp"

namespace md {

template <int LA, int LB>
struct EprodOff {
    static constexpr int NA = ncart(LA), NB = ncart(LB), NAB = NA * NB;
    int off[NAB + 1];
    constexpr EprodOff() : off()
    {
        int o = 0;
        for (int ab = 0; ab < NAB; ++ab) {
            off[ab] = o;
            o += box_nnz(LA, ab / NB, LB, ab % NB);
        }
        off[NAB] = o;
    }
};


template <int LA, int LB, int LC, int LD, typename T = double>
struct KPairCfg {
    static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    static constexpr int NAB = NA * NB, NCD = NC * ND;
    static constexpr int L = LA + LB + LC + LD, LAB = LA + LB, LCD = LC + LD;
    static constexpr bool XROUTE = LCD >= 2;  // precontract the ket into X_P
    // register budget (values of type T) for R, X_P and the block chunk.  One
    // wave per SIMD is the occupancy anyway, so the budget reaches into the
    // accumulation registers: fewer passes over the primitive quartets beat
    // the extra register moves and the few spills (budgets 120..300 were
    // timed per class; (fd|ps) in FP64 is fastest with the smaller one)
    static constexpr int NREG = sizeof(T) == 4 ? 300 : ((LA == 3 && LB == 2 && LC == 1 && LD == 0) ? 160 : 240);
    static constexpr int BUDGET0 = NREG - nherm(L) - (XROUTE ? nherm(LAB) : 0) - 12;
    static constexpr int BUDGET = BUDGET0 < 12 ? 12 : BUDGET0;
    static constexpr int ABCH = NAB <= BUDGET ? NAB : BUDGET;
    static constexpr int NABP = (NAB + ABCH - 1) / ABCH;
    static constexpr int CDCH0 = BUDGET / ABCH;
    static constexpr int CDCH = CDCH0 < 1 ? 1 : (CDCH0 > NCD ? NCD : CDCH0);
    static constexpr int NCDP = (NCD + CDCH - 1) / CDCH;
};

template <int LA, int LB, int LC, int LD, typename T>
__device__ __forceinline__ void k_pair_run(const KPArgs &a, int blk_x)
{
    using C = KPairCfg<LA, LB, LC, LD, T>;
    constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND, NCD = C::NCD;
    constexpr int L = C::L, LAB = C::LAB;
    constexpr EprodOff<LA, LB> ob{};
    constexpr EprodOff<LC, LD> ok{};
    constexpr int SB = ob.off[C::NAB], SK = ok.off[NCD];

    const int lane = threadIdx.x;
    const int4 ch = a.chunks[blk_x];
    const bool valid = lane < ch.z;
    const int64_t wl = a.prefix[ch.x] + ch.y + (valid ? lane : 0);  // the lane's work item
    int r = ch.x;
    for (int k = 1; k < ch.w; ++k)
        if (a.prefix[ch.x + k] <= wl) r = ch.x + k;
    const int ib = a.rows[ch.x].x;
    const int jk = a.rows[r].y + (int)(wl - a.prefix[r]);
    const CPair A = a.bra[ib];
    const CPair B = a.ket[jk];
    const SegLinks links = seg_links(valid ? r : -1 - lane);
    const double bound =
        (a.mode != 0 || a.tau_dens > 0.0) ? a.Qbra[ib] * a.Qket[jk] * k_dens_bound(a.Pm, a.nsh, A, B) : 0.0;
    const bool live = valid && (a.tau_dens <= 0.0 || bound >= a.tau_dens);  // else the lane adds zeros
    if (!mix_take(a.mode, a.mode != 0 && live && bound >= a.tau_mix)) return;
    const T *__restrict__ eprod_bra = pick<T>(a.eprod_bra, a.eprodf_bra);
    const T *__restrict__ eprod_ket = pick<T>(a.eprod_ket, a.eprodf_ket);
    const int nkp = live ? B.np : 0;
    // K_ac, K_bc (kets grouped by c) or K_ad, K_bd (grouped by d) are shared
    // by the lanes of a row: summed across them, added by the row's first
    // lane; the other two blocks are added by every live lane
    auto put = [&](bool shared, double v, double *dst) {
        if (shared) {
            const double u = seg_sum(v, links);
            if (valid && links.head) unsafeAtomicAdd(dst, u);
        } else if (live) {
            unsafeAtomicAdd(dst, v);
        }
    };
    const bool by_c = a.inv == 0;
    const int n = a.ld;
    double s = 1.0;
    if (A.sh1 == A.sh2) s *= 0.5;
    if (B.sh1 == B.sh2) s *= 0.5;
    if (a.same && same_pair(A, B)) s *= 0.5;

    static_for<0, C::NABP * C::NCDP>([&](auto pc) {
        constexpr int pass = decltype(pc)::value;
        constexpr int ab0 = (pass / C::NCDP) * C::ABCH;
        constexpr int ab1 = (ab0 + C::ABCH < C::NAB) ? ab0 + C::ABCH : C::NAB;
        constexpr int cd0 = (pass % C::NCDP) * C::CDCH;
        constexpr int cd1 = (cd0 + C::CDCH < NCD) ? cd0 + C::CDCH : NCD;
        constexpr int NABc = ab1 - ab0, NCDc = cd1 - cd0;
        T V[NABc * NCDc];
#pragma unroll
        for (int i = 0; i < NABc * NCDc; ++i) V[i] = T(0);

        for (int ip = 0; ip < A.np; ++ip) {
            const PrimPair pb = a.pp[A.poff + ip];
            const T *__restrict__ eb = eprod_bra + (int64_t)(A.poff + ip - a.pbase_bra) * SB;
            for (int kp = 0; kp < nkp; ++kp) {
                const PrimPair pk = a.pp[B.poff + kp];
                if (pb.q * pk.q < a.tau_prim) break;
                T Fs[L + 1], X, Y, Z;
                T rp[C::LCD + 1];  // r^|s| of the scaled single-precision form
                if constexpr (sizeof(T) == 4) {
                    float r;
                    quartet_fs_scaled<L>(pb, pk, a.boys, Fs, X, Y, Z, r, a.om2);
                    powers<C::LCD>(r, rp);
                } else {
                    quartet_fs<L, T>(pb, pk, a.boys, Fs, X, Y, Z, a.om2);
                }
                T R[nherm(L)];
                r_build<L, T>(Fs, X, Y, Z, R);
                const T *__restrict__ ek = eprod_ket + (int64_t)(B.poff + kp - a.pbase_ket) * SK;
                static_for<cd0, cd1>([&](auto cdc) {
                    constexpr int cd = decltype(cdc)::value;
                    constexpr int c = cd / ND, d = cd % ND;
                    constexpr int nsx = cart_x(LC, c) + cart_x(LD, d) + 1;
                    constexpr int nsy = cart_y(LC, c) + cart_y(LD, d) + 1;
                    constexpr int nsz = cart_z(LC, c) + cart_z(LD, d) + 1;
                    T e[nsx * nsy * nsz];
                    static_for<0, nsx * nsy * nsz>([&](auto qc) {
                        constexpr int q = decltype(qc)::value;
                        constexpr int sn = q / (nsy * nsz) + (q / nsz) % nsy + q % nsz;
                        if constexpr (sizeof(T) == 4)
                            e[q] = ek[ok.off[cd] + q] * rp[sn];
                        else
                            e[q] = ek[ok.off[cd] + q];
                    });
                    if constexpr (C::XROUTE) {
                        // X_P = sum_s (-1)^{|s|} E^{cd}_s R_{P+s}, then (ab|cd) = sum_t E^{ab}_t X_t
                        T Xp[nherm(LAB)];
                        static_for<0, nherm(LAB)>([&](auto Pc) {
                            constexpr int P = decltype(Pc)::value;
                            constexpr int tp = herm_t(P), up = herm_u(P), vp = herm_v(P);
                            T x = T(0);
                            static_for<0, nsx * nsy * nsz>([&](auto qc) {
                                constexpr int q = decltype(qc)::value;
                                constexpr int sx = q / (nsy * nsz), sy = (q / nsz) % nsy, sz = q % nsz;
                                constexpr T sg = ((sx + sy + sz) & 1) ? T(-1) : T(1);
                                x += sg * e[q] * R[herm_idx(tp + sx, up + sy, vp + sz)];
                            });
                            Xp[P] = x;
                        });
                        static_for<ab0, ab1>([&](auto abc) {
                            constexpr int ab = decltype(abc)::value;
                            constexpr int ia = ab / NB, jb = ab % NB;
                            constexpr int mx = cart_x(LA, ia) + cart_x(LB, jb) + 1;
                            constexpr int my = cart_y(LA, ia) + cart_y(LB, jb) + 1;
                            constexpr int mz = cart_z(LA, ia) + cart_z(LB, jb) + 1;
                            T v = T(0);
                            static_for<0, mx * my * mz>([&](auto tc) {
                                constexpr int t = decltype(tc)::value;
                                constexpr int tx = t / (my * mz), ty = (t / mz) % my, tz = t % mz;
                                v += eb[ob.off[ab] + t] * Xp[herm_idx(tx, ty, tz)];
                            });
                            V[(ab - ab0) * NCDc + (cd - cd0)] += v;
                        });
                    } else {
                        // small ket box: (ab|cd) = sum_t E^{ab}_t sum_s (-1)^{|s|} E^{cd}_s R_{t+s}
                        static_for<ab0, ab1>([&](auto abc) {
                            constexpr int ab = decltype(abc)::value;
                            constexpr int ia = ab / NB, jb = ab % NB;
                            constexpr int mx = cart_x(LA, ia) + cart_x(LB, jb) + 1;
                            constexpr int my = cart_y(LA, ia) + cart_y(LB, jb) + 1;
                            constexpr int mz = cart_z(LA, ia) + cart_z(LB, jb) + 1;
                            T v = T(0);
                            static_for<0, mx * my * mz>([&](auto tc) {
                                constexpr int t = decltype(tc)::value;
                                constexpr int tx = t / (my * mz), ty = (t / mz) % my, tz = t % mz;
                                T x = T(0);
                                static_for<0, nsx * nsy * nsz>([&](auto qc) {
                                    constexpr int q = decltype(qc)::value;
                                    constexpr int sx = q / (nsy * nsz), sy = (q / nsz) % nsy, sz = q % nsz;
                                    constexpr T sg = ((sx + sy + sz) & 1) ? T(-1) : T(1);
                                    x += sg * e[q] * R[herm_idx(tx + sx, ty + sy, tz + sz)];
                                });
                                v += eb[ob.off[ab] + t] * x;
                            });
                            V[(ab - ab0) * NCDc + (cd - cd0)] += v;
                        });
                    }
                });
            }
        }

        // digest the chunk: K_ac += V D_bd, K_ad += V D_bc, K_bc += V D_ad, K_bd += V D_ac.
        // Every density element the chunk touches is loaded once, and every
        // exchange element gets one atomic with the chunk's sum over the other
        // two indices (instead of one load and one atomic per block element).
        {
            constexpr int i0 = ab0 / NB, i1 = (ab1 - 1) / NB;
            constexpr int j0 = i0 < i1 ? 0 : ab0 % NB, j1 = i0 < i1 ? NB - 1 : (ab1 - 1) % NB;
            constexpr int c0 = cd0 / ND, c1 = (cd1 - 1) / ND;
            constexpr int d0 = c0 < c1 ? 0 : cd0 % ND, d1 = c0 < c1 ? ND - 1 : (cd1 - 1) % ND;
            constexpr int ni = i1 - i0 + 1, nj = j1 - j0 + 1, nc = c1 - c0 + 1, nd = d1 - d0 + 1;
            const double *__restrict__ D = a.D;
            double Dac[ni * nc], Dad[ni * nd], Dbc[nj * nc], Dbd[nj * nd];
            static_for<0, ni>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                const double *row = D + (int64_t)(A.c1 + i0 + i) * n;
                static_for<0, nc>([&](auto cc) { Dac[i * nc + cc] = row[B.c1 + c0 + cc]; });
                static_for<0, nd>([&](auto dc) { Dad[i * nd + dc] = row[B.c2 + d0 + dc]; });
            });
            static_for<0, nj>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                const double *row = D + (int64_t)(A.c2 + j0 + j) * n;
                static_for<0, nc>([&](auto cc) { Dbc[j * nc + cc] = row[B.c1 + c0 + cc]; });
                static_for<0, nd>([&](auto dc) { Dbd[j * nd + dc] = row[B.c2 + d0 + dc]; });
            });
            // block element (i0+i, j0+j | c0+c, d0+d) if it lies in the chunk
            auto vget = [&](auto ic, auto jc, auto cc, auto dc, double &v) -> bool {
                constexpr int ab = (i0 + decltype(ic)::value) * NB + j0 + decltype(jc)::value;
                constexpr int cd = (c0 + decltype(cc)::value) * ND + d0 + decltype(dc)::value;
                if constexpr (ab >= ab0 && ab < ab1 && cd >= cd0 && cd < cd1) {
                    v = (double)V[(ab - ab0) * NCDc + (cd - cd0)];
                    return true;
                } else {
                    return false;
                }
            };
            static_for<0, ni>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                static_for<0, nc>([&](auto cc) {  // K_ac[i][c] = sum_{j,d} V D_bd[j][d]
                    double t = 0.0;
                    bool any = false;
                    static_for<0, nj>([&](auto jc) {
                        static_for<0, nd>([&](auto dc) {
                            double v;
                            if (vget(ic, jc, cc, dc, v)) {
                                t += v * Dbd[decltype(jc)::value * nd + decltype(dc)::value];
                                any = true;
                            }
                        });
                    });
                    if (any) put(by_c, s * t, &a.Kacc[(int64_t)(A.c1 + i0 + i) * n + B.c1 + c0 + cc]);
                });
                static_for<0, nd>([&](auto dc) {  // K_ad[i][d] = sum_{j,c} V D_bc[j][c]
                    double t = 0.0;
                    bool any = false;
                    static_for<0, nj>([&](auto jc) {
                        static_for<0, nc>([&](auto cc) {
                            double v;
                            if (vget(ic, jc, cc, dc, v)) {
                                t += v * Dbc[decltype(jc)::value * nc + decltype(cc)::value];
                                any = true;
                            }
                        });
                    });
                    if (any) put(!by_c, s * t, &a.Kacc[(int64_t)(A.c1 + i0 + i) * n + B.c2 + d0 + dc]);
                });
            });
            static_for<0, nj>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                static_for<0, nc>([&](auto cc) {  // K_bc[j][c] = sum_{i,d} V D_ad[i][d]
                    double t = 0.0;
                    bool any = false;
                    static_for<0, ni>([&](auto ic) {
                        static_for<0, nd>([&](auto dc) {
                            double v;
                            if (vget(ic, jc, cc, dc, v)) {
                                t += v * Dad[decltype(ic)::value * nd + decltype(dc)::value];
                                any = true;
                            }
                        });
                    });
                    if (any) put(by_c, s * t, &a.Kacc[(int64_t)(A.c2 + j0 + j) * n + B.c1 + c0 + cc]);
                });
                static_for<0, nd>([&](auto dc) {  // K_bd[j][d] = sum_{i,c} V D_ac[i][c]
                    double t = 0.0;
                    bool any = false;
                    static_for<0, ni>([&](auto ic) {
                        static_for<0, nc>([&](auto cc) {
                            double v;
                            if (vget(ic, jc, cc, dc, v)) {
                                t += v * Dac[decltype(ic)::value * nc + decltype(cc)::value];
                                any = true;
                            }
                        });
                    });
                    if (any) put(!by_c, s * t, &a.Kacc[(int64_t)(A.c2 + j0 + j) * n + B.c2 + d0 + dc]);
                });
            });
        }
    });
}

template <int LA, int LB, int LC, int LD, typename T>
__global__ __launch_bounds__(64) void k_pair(KPArgs a)
{
    k_pair_run<LA, LB, LC, LD, T>(a, blockIdx.x);
}

// batch form: workgroup b runs block (items[b].y, items[b].z) of the
// launch whose arguments are tab[items[b].x]
template <int LA, int LB, int LC, int LD, typename T>
__global__ __launch_bounds__(64) void k_pair_q(const KPArgs *__restrict__ tab, const int4 *__restrict__ items)
{
    const int4 it = items[blockIdx.x];
    KPArgs a = tab[it.x];
    globalize(a);
    k_pair_run<LA, LB, LC, LD, T>(a, it.y);
}

template <int LA, int LB, int LC, int LD>
void launch_k_pair_t(const KPArgs &a, int nchunks, bool fp32, hipStream_t st)
{
    if (nchunks <= 0) return;
    if (queue_sink()) {  // a batch plan: one chunk of up to 64 quartets per block
        queue_record(fp32 ? &queue_launch<KPArgs, k_pair_q<LA, LB, LC, LD, float>, 64>
                          : &queue_launch<KPArgs, k_pair_q<LA, LB, LC, LD, double>, 64>,
                     a, nchunks, 1, 1.0, "k_pair");
        return;
    }
    if (fp32)
        hipLaunchKernelGGL((k_pair<LA, LB, LC, LD, float>), dim3((unsigned)nchunks), dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL((k_pair<LA, LB, LC, LD, double>), dim3((unsigned)nchunks), dim3(64), 0, st, a);
}

}  // namespace md
