// k_small.hip -- exchange (K) for angular classes whose Cartesian block fits
// in registers: one lane evaluates one canonical contracted shell quartet,
// looping over its primitive quartets (eq. eri_formula with E built in-kernel),
// accumulates the contracted Cartesian block and digests it into the four
// exchange blocks that the 8-fold permutational symmetry (eq. 8_fold_symmetry)
// maps it to:  K_ac += V D_bd, K_ad += V D_bc, K_bc += V D_ad, K_bd += V D_ac.
// Neighbouring lanes of one work-list row share the bra and one ket shell
// (c, or d in the grouping that the paper calls inverted), so their K_ac and
// K_bc (or K_ad and K_bd) terms are summed across the lanes before one
// atomic addition per element.  A density-weighted screen may skip lanes.
// The caller forms K = Kacc + Kacc^T afterwards.  T is the arithmetic type of
// the primitive integrals; the digestion and the accumulator stay in double
// precision.  In the mixed mode a wavefront (64 consecutive quartets) is one
// precision tile.
#include "class_lists.hpp"
#include "kern_args.hpp"
#include "md_device.hpp"
#include "queue.hpp"

namespace md {

template <int LA, int LB, int LC, int LD, typename T>
__device__ __forceinline__ void k_small_run(const KArgs &a, int blk_x)
{
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int L = LA + LB + LC + LD, LAB = LA + LB;
    constexpr int NBLK = NA * NB * NC * ND;
    constexpr bool F32 = sizeof(T) == 4;

    // every lane of a wavefront stays to the end (the digestion sums across
    // lanes); lanes past the work list evaluate nothing
    const int64_t w = (int64_t)blk_x * 128 + threadIdx.x;
    const bool valid = w < a.nwork;
    const int64_t wc = valid ? w : a.nwork - 1;
    const int r = k_find_row(a.prefix, a.nrows, wc);
    const int2 rw = a.rows[r];
    const int ib = rw.x;
    const int jk = rw.y + (int)(wc - a.prefix[r]);
    const CPair A = a.bra[ib];
    const CPair B = a.ket[jk];
    // a live lane evaluates its quartet; the others (past the work list, or
    // below the density-weighted screen) contribute zeros
    const double bound =
        (a.mode != 0 || a.tau_dens > 0.0) ? a.Qbra[ib] * a.Qket[jk] * k_dens_bound(a.Pm, a.nsh, A, B) : 0.0;
    const bool live = valid && (a.tau_dens <= 0.0 || bound >= a.tau_dens);
    if (!mix_take(a.mode, a.mode != 0 && live && bound >= a.tau_mix)) return;  // uniform over the wavefront
    const int nbp = live ? A.np : 0;

    T V[NBLK];
#pragma unroll
    for (int i = 0; i < NBLK; ++i) V[i] = T(0);

    const double qk0 = a.pp[B.poff].q;
    for (int ip = 0; ip < nbp; ++ip) {
        const PrimPair pb = a.pp[A.poff + ip];
        if (pb.q * qk0 < a.tau_prim) break;
        Etab<LA, LB, T> Ex, Ey, Ez;
        etab_build<LA, LB, T>((T)pb.PA[0], (T)pb.PB[0], (T)pb.o2p, Ex);
        etab_build<LA, LB, T>((T)pb.PA[1], (T)pb.PB[1], (T)pb.o2p, Ey);
        etab_build<LA, LB, T>((T)pb.PA[2], (T)pb.PB[2], (T)pb.o2p, Ez);
        float cb = 0.f;
        if constexpr (F32) {  // scaled single-precision form (md_device.hpp)
            cb = (float)sqrt(2.0 * pb.p);
            etab_scale<LA, LB>(Ex, cb, (float)pb.K);
            etab_scale<LA, LB>(Ey, cb, 1.f);
            etab_scale<LA, LB>(Ez, cb, 1.f);
        }
        for (int kp = 0; kp < B.np; ++kp) {
            const PrimPair pk = a.pp[B.poff + kp];
            if (pb.q * pk.q < a.tau_prim) break;
            T Fs[L + 1], X, Y, Z;
            if constexpr (F32) {
                float r;
                quartet_fs_scaled<L>(pb, pk, a.boys, Fs, X, Y, Z, r, a.om2);
            } else {
                quartet_fs<L, T>(pb, pk, a.boys, Fs, X, Y, Z, a.om2);
            }
            T R[nherm(L)];
            r_build<L, T>(Fs, X, Y, Z, R);
            Etab<LC, LD, T> Fx, Fy, Fz;
            etab_build<LC, LD, T>((T)pk.PA[0], (T)pk.PB[0], (T)pk.o2p, Fx);
            etab_build<LC, LD, T>((T)pk.PA[1], (T)pk.PB[1], (T)pk.o2p, Fy);
            etab_build<LC, LD, T>((T)pk.PA[2], (T)pk.PB[2], (T)pk.o2p, Fz);
            if constexpr (F32) {  // ket factors carry the bra's c
                etab_scale<LC, LD>(Fx, cb, (float)pk.K);
                etab_scale<LC, LD>(Fy, cb, 1.f);
                etab_scale<LC, LD>(Fz, cb, 1.f);
            }
            static_for<0, NC * ND>([&](auto cdc) {
                constexpr int cd = decltype(cdc)::value;
                constexpr int c = cd / ND, d = cd % ND;
                constexpr int cx = cart_x(LC, c), cy = cart_y(LC, c), cz = cart_z(LC, c);
                constexpr int dx = cart_x(LD, d), dy = cart_y(LD, d), dz = cart_z(LD, d);
                // X_P = sum_s (-1)^{|s|} E^{cd}_s R_{P+s}   (ket half of eq. eri_formula)
                T Xp[nherm(LAB)];
                static_for<0, nherm(LAB)>([&](auto pc) {
                    constexpr int P = decltype(pc)::value;
                    constexpr int tp = herm_t(P), up = herm_u(P), vp = herm_v(P);
                    T s = T(0);
                    static_for<0, cx + dx + 1>([&](auto sxc) {
                        constexpr int sx = decltype(sxc)::value;
                        static_for<0, cy + dy + 1>([&](auto syc) {
                            constexpr int sy = decltype(syc)::value;
                            const T exy = Fx.e[cx][dx][sx] * Fy.e[cy][dy][sy];
                            static_for<0, cz + dz + 1>([&](auto szc) {
                                constexpr int sz = decltype(szc)::value;
                                constexpr T sg = ((sx + sy + sz) & 1) ? T(-1) : T(1);
                                s += sg * exy * Fz.e[cz][dz][sz] * R[herm_idx(tp + sx, up + sy, vp + sz)];
                            });
                        });
                    });
                    Xp[P] = s;
                });
                // (ab|cd) += sum_P E^{ab}_P X_P
                static_for<0, NA * NB>([&](auto abc) {
                    constexpr int ab = decltype(abc)::value;
                    constexpr int ia = ab / NB, jb = ab % NB;
                    constexpr int ax = cart_x(LA, ia), ay = cart_y(LA, ia), az = cart_z(LA, ia);
                    constexpr int bx = cart_x(LB, jb), by = cart_y(LB, jb), bz = cart_z(LB, jb);
                    T v = T(0);
                    static_for<0, ax + bx + 1>([&](auto txc) {
                        constexpr int tx = decltype(txc)::value;
                        static_for<0, ay + by + 1>([&](auto tyc) {
                            constexpr int ty = decltype(tyc)::value;
                            const T exy = Ex.e[ax][bx][tx] * Ey.e[ay][by][ty];
                            static_for<0, az + bz + 1>([&](auto tzc) {
                                constexpr int tz = decltype(tzc)::value;
                                v += exy * Ez.e[az][bz][tz] * Xp[herm_idx(tx, ty, tz)];
                            });
                        });
                    });
                    V[ab * (NC * ND) + cd] += v;
                });
            });
        }
    }

    // degeneracy of the canonical quartet
    double s = 1.0;
    if (A.sh1 == A.sh2) s *= 0.5;
    if (B.sh1 == B.sh2) s *= 0.5;
    if (a.same && same_pair(A, B)) s *= 0.5;

    // Each density element is loaded once: the loads could not otherwise be
    // hoisted past the atomics, and every block element would reload two.
    // K_ac and K_bc of the lanes of one row (same bra, same ket shell c) are
    // summed across those lanes and added once by the row's first lane;
    // K_ad and K_bd are added by every lane.
    const double *__restrict__ D = a.D;
    const int n = a.ld;
    double *Kc = a.Kacc;
    double kac[NA * NC], kad[NA * ND], kbc[NB * NC], kbd[NB * ND];
    {  // K_ac = V D_bd and K_ad = V D_bc (density rows of the second bra shell)
        double Dbd[NB * ND], Dbc[NB * NC];
        static_for<0, NB>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const double *row = D + (int64_t)(A.c2 + j) * n;
            static_for<0, ND>([&](auto lc) { Dbd[j * ND + lc] = row[B.c2 + lc]; });
            static_for<0, NC>([&](auto kc) { Dbc[j * NC + kc] = row[B.c1 + kc]; });
        });
        static_for<0, NA>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            static_for<0, NC>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                double acc = 0.0;
                static_for<0, NB>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    static_for<0, ND>([&](auto lc) {
                        constexpr int l = decltype(lc)::value;
                        acc += (double)V[((i * NB + j) * NC + k) * ND + l] * Dbd[j * ND + l];
                    });
                });
                kac[i * NC + k] = s * acc;
            });
            static_for<0, ND>([&](auto lc) {
                constexpr int l = decltype(lc)::value;
                double acc = 0.0;
                static_for<0, NB>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    static_for<0, NC>([&](auto kc) {
                        constexpr int k = decltype(kc)::value;
                        acc += (double)V[((i * NB + j) * NC + k) * ND + l] * Dbc[j * NC + k];
                    });
                });
                kad[i * ND + l] = s * acc;
            });
        });
    }
    {  // K_bc = V D_ad and K_bd = V D_ac, one density row of the first bra shell at a time
#pragma unroll
        for (int o = 0; o < NB * NC; ++o) kbc[o] = 0.0;
#pragma unroll
        for (int o = 0; o < NB * ND; ++o) kbd[o] = 0.0;
        static_for<0, NA>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const double *row = D + (int64_t)(A.c1 + i) * n;
            double Dad[ND], Dac[NC];
            static_for<0, ND>([&](auto lc) { Dad[lc] = row[B.c2 + lc]; });
            static_for<0, NC>([&](auto kc) { Dac[kc] = row[B.c1 + kc]; });
            static_for<0, NB>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                static_for<0, NC>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    static_for<0, ND>([&](auto lc) {
                        constexpr int l = decltype(lc)::value;
                        const double v = (double)V[((i * NB + j) * NC + k) * ND + l];
                        kbc[j * NC + k] += v * Dad[l];
                        kbd[j * ND + l] += v * Dac[k];
                    });
                });
            });
        });
    }
    // The two blocks whose targets the lanes of a row share (K_ac, K_bc when
    // the kets are grouped by c; K_ad, K_bd when grouped by d) are summed
    // across those lanes and added by the row's first lane (a skipped lane
    // adds zeros, so it may lead its row); the other two by every live lane.
    const SegLinks links = seg_links(valid ? r : -1 - (int)(threadIdx.x & 63));
    if (!a.inv) {
        static_for<0, NA * NC>([&](auto oc) {
            constexpr int o = decltype(oc)::value;
            const double v = seg_sum(kac[o], links);
            if (valid && links.head) unsafeAtomicAdd(&Kc[(int64_t)(A.c1 + o / NC) * n + B.c1 + o % NC], v);
        });
        static_for<0, NB * NC>([&](auto oc) {
            constexpr int o = decltype(oc)::value;
            const double v = seg_sum(s * kbc[o], links);
            if (valid && links.head) unsafeAtomicAdd(&Kc[(int64_t)(A.c2 + o / NC) * n + B.c1 + o % NC], v);
        });
        if (live) {
            static_for<0, NA * ND>([&](auto oc) {
                constexpr int o = decltype(oc)::value;
                unsafeAtomicAdd(&Kc[(int64_t)(A.c1 + o / ND) * n + B.c2 + o % ND], kad[o]);
            });
            static_for<0, NB * ND>([&](auto oc) {
                constexpr int o = decltype(oc)::value;
                unsafeAtomicAdd(&Kc[(int64_t)(A.c2 + o / ND) * n + B.c2 + o % ND], s * kbd[o]);
            });
        }
    } else {
        static_for<0, NA * ND>([&](auto oc) {
            constexpr int o = decltype(oc)::value;
            const double v = seg_sum(kad[o], links);
            if (valid && links.head) unsafeAtomicAdd(&Kc[(int64_t)(A.c1 + o / ND) * n + B.c2 + o % ND], v);
        });
        static_for<0, NB * ND>([&](auto oc) {
            constexpr int o = decltype(oc)::value;
            const double v = seg_sum(s * kbd[o], links);
            if (valid && links.head) unsafeAtomicAdd(&Kc[(int64_t)(A.c2 + o / ND) * n + B.c2 + o % ND], v);
        });
        if (live) {
            static_for<0, NA * NC>([&](auto oc) {
                constexpr int o = decltype(oc)::value;
                unsafeAtomicAdd(&Kc[(int64_t)(A.c1 + o / NC) * n + B.c1 + o % NC], kac[o]);
            });
            static_for<0, NB * NC>([&](auto oc) {
                constexpr int o = decltype(oc)::value;
                unsafeAtomicAdd(&Kc[(int64_t)(A.c2 + o / NC) * n + B.c1 + o % NC], s * kbc[o]);
            });
        }
    }
}

template <int LA, int LB, int LC, int LD, typename T>
__global__ __launch_bounds__(128) void k_small(KArgs a)
{
    k_small_run<LA, LB, LC, LD, T>(a, blockIdx.x);
}

// batch form: workgroup b runs block (items[b].y, items[b].z) of the
// launch whose arguments are tab[items[b].x]
template <int LA, int LB, int LC, int LD, typename T>
__global__ __launch_bounds__(128) void k_small_q(const KArgs *__restrict__ tab, const int4 *__restrict__ items)
{
    const int4 it = items[blockIdx.x];
    KArgs a = tab[it.x];
    globalize(a);
    k_small_run<LA, LB, LC, LD, T>(a, it.y);
}

bool launch_k_small(int la, int lb, int lc, int ld, const KArgs &a, bool fp32, hipStream_t st)
{
    const int threads = 128;
    const int64_t blocks = (a.nwork + threads - 1) / threads;
    if (a.nwork <= 0) return true;
#define MD_CASE(A_, B_, C_, D_)                                                        \
    if (la == A_ && lb == B_ && lc == C_ && ld == D_) {                                \
        if (queue_sink())                                                              \
            queue_record(fp32 ? &queue_launch<KArgs, k_small_q<A_, B_, C_, D_, float>, 128>             \
                              : &queue_launch<KArgs, k_small_q<A_, B_, C_, D_, double>, 128>,            \
                         a, (int)blocks, 1, 1.0,                                       \
                         "k_small");                                                   \
        else if (fp32)                                                                 \
            hipLaunchKernelGGL((k_small<A_, B_, C_, D_, float>), dim3((unsigned)blocks), dim3(threads), 0, st, a); \
        else                                                                           \
            hipLaunchKernelGGL((k_small<A_, B_, C_, D_, double>), dim3((unsigned)blocks), dim3(threads), 0, st, a); \
        return true;                                                                   \
    }
    MD_K_SMALL_LIST(MD_CASE)
#undef MD_CASE
    return false;
}

}  // namespace md
