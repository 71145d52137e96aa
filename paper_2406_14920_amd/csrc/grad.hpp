// grad.hpp -- nuclear gradient of E = 1/2 tr(PJ) - 1/4 tr(PK) at fixed P
// (SI eqs. si_E_J_K, si_dE_J, si_dE_K).
//
// Derivative of a primitive pair with respect to its first centre (the
// content of SI eq. si_pair_derivative, written with the Gaussian identity
// d/dA_x x_A^i e^{-a x_A^2} = 2a x_A^{i+1} e^{..} - i x_A^{i-1} e^{..}):
//     d/dA_k (ab) = sum_t Ed^{A,k}_t Lambda_t,
//     Ed^{A,k} = (2a E^{i_k+1, j_k} - i_k E^{i_k-1, j_k}) along k, E^{ij} along the others,
// and, because the Hermite Gaussians depend on A and B only through P,
//     (d/dA_k + d/dB_k)(ab) = sum_t E_t Lambda_{t+1_k}.
// So a derivative needs the Hermite index one higher than the integral
// (R up to L+1), and dB = (dA + dB) - dA.
//
// Exchange part (eq. si_dE_K over all centres of a canonical quartet,
// weights of the 8-fold orbit): per canonical quartet
//     W_{ab,cd} = -s (D_ac D_bd + D_ad D_bc),
//     g_A = sum W d_A(ab|cd),  g_S = sum W (d_A + d_B)(ab|cd),  g_C = sum W d_C(ab|cd),
//     g_B = g_S - g_A,  g_D = -g_S - g_C  (translational invariance).
// One 64-lane workgroup per quartet: per primitive quartet R^0 up to L+1 goes
// to LDS, the ket-contracted intermediates
//     X^{cd}_t   = sum_s (-1)^{|s|} E^{cd}_s R_{t+s},          t in H(LAB+1)
//     Xc^{cd,k}_t = sum_s (-1)^{|s|} Ed^{C,k}_{cd,s} R_{t+s},  t in H(LAB)
// are built cooperatively for a chunk of ket components, and lane ab
// contracts them with its bra coefficients and the weights (when one chunk
// holds every ket component the intermediates are first summed over the ket
// primitive pairs, so the contraction runs once per bra primitive pair).  Gradient
// contributions are summed per workgroup in LDS by one lane in work order and
// written as per-workgroup partials, which a final kernel adds in a fixed
// order (deterministic).
#pragma once
#include "class_lists.hpp"
#include "kern_args.hpp"
#include "launch.hpp"
#include "md_device.hpp"
#include "wave_r.hpp"

namespace md {

// largest Hermite box of a pair class with one axis extended by one (the
// derivative boxes), over all components and axes
__host__ __device__ constexpr int box_max_ext(int la, int lb)
{
    int m = 0;
    for (int ca = 0; ca < ncart(la); ++ca)
        for (int cb = 0; cb < ncart(lb); ++cb) {
            const int nx = cart_x(la, ca) + cart_x(lb, cb) + 1, ny = cart_y(la, ca) + cart_y(lb, cb) + 1,
                      nz = cart_z(la, ca) + cart_z(lb, cb) + 1;
            const int v = (nx + 1) * ny * nz > nx * (ny + 1) * nz ? (nx + 1) * ny * nz : nx * (ny + 1) * nz;
            const int w = v > nx * ny * (nz + 1) ? v : nx * ny * (nz + 1);
            if (w > m) m = w;
        }
    return m;
}

// largest Hermite box of a pair class grown by one along every axis
__host__ __device__ constexpr int box_max_grown(int la, int lb)
{
    int m = 0;
    for (int ca = 0; ca < ncart(la); ++ca)
        for (int cb = 0; cb < ncart(lb); ++cb) {
            const int v = (cart_x(la, ca) + cart_x(lb, cb) + 2) * (cart_y(la, ca) + cart_y(lb, cb) + 2) *
                          (cart_z(la, ca) + cart_z(lb, cb) + 2);
            if (v > m) m = v;
        }
    return m;
}

// LDS bytes of kg_wave's tables with a ket chunk of c components (the
// natom x 3 partials come on top)
__host__ __device__ constexpr int kg_lds_bytes(int L, int NR0, int EBD, int EKD, int NHX, int NHC, int ND_, int KBM,
                                               int c)
{
    return 8 * (NR0 + (L + 2) + 3 * (L + 2) * ((L + 1) / 2 + 1) + 3 * EBD + 3 * EKD + c * NHX + 3 * c * NHC + ND_) +
           4 * nherm(L + 1) + 12 * 4 * c * KBM;
}

template <int LA, int LB, int LC, int LD>
struct KGCfg {
    static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    static constexpr int NAB = NA * NB, NCD = NC * ND;
    static constexpr int L = LA + LB + LC + LD, LAB = LA + LB, LCD = LC + LD;
    static constexpr int L2 = L + 2;                 // dense R table side (orders up to L+1)
    static constexpr int NR0 = L2 * L2 * L2;
    static constexpr int NHX = nherm(LAB + 1), NHC = nherm(LAB);
    static constexpr int NABCH = (NAB + 63) / 64;
    // 1D tables [i][j][t]: bra i <= LA+1, j <= LB, t <= LAB+1; ket i <= LC+1, j <= LD, t <= LCD+1
    static constexpr int EBJ = LAB + 2, EBI = (LB + 1) * EBJ, EBD = (LA + 2) * EBI;
    static constexpr int EKJ = LCD + 2, EKI = (LD + 1) * EKJ, EKD = (LC + 2) * EKI;
    static constexpr int ND_ = NA * NC + NA * ND + NB * NC + NB * ND;
    static constexpr int KBM = box_max_ext(LC, LD);  // longest ket coefficient list
    // ket components per chunk: all of them (up to 24) if their tables fit in
    // 48 KB of LDS (three workgroups per compute unit; one chunk lets the
    // intermediates be summed over the ket primitive pairs, worth more than
    // the fourth workgroup), else the largest of 16, 8, 4 whose tables fit in
    // 40 KB, so that four of these one-wave workgroups share a compute unit
    // (one per SIMD; the largest classes hold 256 VGPRs, one wave per SIMD)
    static constexpr bool ALL = NCD <= 24 && kg_lds_bytes(L, NR0, EBD, EKD, NHX, NHC, ND_, KBM, NCD) <= 49152;
    static constexpr int CDCH0 = ALL ? NCD
                                 : kg_lds_bytes(L, NR0, EBD, EKD, NHX, NHC, ND_, KBM, 16) <= 40960 ? 16
                                 : kg_lds_bytes(L, NR0, EBD, EKD, NHX, NHC, ND_, KBM, 8) <= 40960  ? 8
                                                                                                   : 4;
    static constexpr int CDCH = NCD < CDCH0 ? NCD : CDCH0;
    static constexpr int RANGE = 4;
};

// Derivative coefficient along one axis: 2a E^{i+1,j}_t - i E^{i-1,j}_t.
__device__ __forceinline__ double dcoef(const double *E, int DI, int DJ, int i, int j, int t, double a2)
{
    double v = a2 * E[(i + 1) * DI + j * DJ + t];
    if (i > 0) v -= (double)i * E[(i - 1) * DI + j * DJ + t];
    return v;
}

template <int LA, int LB, int LC, int LD>
__global__ __launch_bounds__(64) void kg_wave(KGArgs g)
{
    using C = KGCfg<LA, LB, LC, LD>;
    constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND, NAB = C::NAB, NCD = C::NCD;
    constexpr int L = C::L, L2 = C::L2, CDCH = C::CDCH, NHX = C::NHX, NHC = C::NHC;
    // all ket components in one chunk: the ket-contracted intermediates are
    // linear in the ket primitive pairs' contributions and the bra terms depend
    // on the bra primitive pair only, so the intermediates are summed over the
    // ket primitive pairs and the bra contraction runs once per bra primitive
    // pair (as the forward kernel's ket-first form does)
    constexpr bool KACC = NCD <= CDCH;
    const KArgs &a = g.k;

    __shared__ double sR0[C::NR0];
    __shared__ double sF[L + 2];
    __shared__ double sH[HPolyDims<L + 1>::N];
    __shared__ int sHerm[nherm(L + 1)];
    __shared__ double sEb[3 * C::EBD];
    __shared__ double sEk[3 * C::EKD];
    __shared__ double sX[CDCH * NHX];
    __shared__ double sXc[3 * CDCH * NHC];
    __shared__ double sD[C::ND_];
    // ket coefficient lists of a chunk, [kq][c][k]: kq 0 the ket E product,
    // kq 1..3 its derivative along x, y, z; coefficient (sign included) and
    // R offset of box point k, zero past the box
    __shared__ double sEc[4 * CDCH * C::KBM];
    __shared__ int sEo[4 * CDCH * C::KBM];
    extern __shared__ double sG[];  // natom x 3

    const int lane = threadIdx.x;
    herm_table_lds(sHerm, nherm(L + 1), lane);
    // per-lane R^0 term plan (orders up to 9), visible after the first
    // barrier; only where it leaves the workgroups per CU that LDS allows
    // unchanged, with 1 KB to spare for the atom partials (at most eight one-wave
    // workgroups are resident anyway)
    constexpr int LDSK = kg_lds_bytes(L, C::NR0, C::EBD, C::EKD, NHX, NHC, C::ND_, C::KBM, CDCH) + 512;
    constexpr int WGK = 163840 / LDSK < 8 ? 163840 / LDSK : 8;
    constexpr bool PLAN = R0Plan<L + 1, double>::OK && 163840 / (LDSK + R0Plan<L + 1, double>::NT * 256 + 1024) >= WGK;
    __shared__ uint32_t sPlan[PLAN ? R0Plan<L + 1, double>::NT * 64 : 1];
    R0Plan<L + 1, double> r0p;
    r0p.code = sPlan;
    if constexpr (PLAN) r0_plan_build<L + 1, double, L2 * L2, L2>(r0p, lane);
    const int na3 = 3 * g.natom;
    for (int o = lane; o < na3; o += 64) sG[o] = 0.0;
    // every entry finite from the start: the chunk loops below run to CDCH
    // with zero weights past the chunk end
    for (int o = lane; o < CDCH * NHX; o += 64) sX[o] = 0.0;
    for (int o = lane; o < 3 * CDCH * NHC; o += 64) sXc[o] = 0.0;

    const int n = a.ld;
    for (int64_t w0 = (int64_t)blockIdx.x * C::RANGE; w0 < a.nwork; w0 += (int64_t)gridDim.x * C::RANGE) {
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
            double sdeg = 1.0;
            if (A.sh1 == A.sh2) sdeg *= 0.5;
            if (B.sh1 == B.sh2) sdeg *= 0.5;
            if (a.same && same_pair(A, B)) sdeg *= 0.5;

            // density tiles D_ac, D_ad, D_bc, D_bd
            for (int o = lane; o < C::ND_; o += 64) {
                int row, col;
                if (o < NA * NC) { row = A.c1 + o / NC; col = B.c1 + o % NC; }
                else if (o < NA * NC + NA * ND) { int r = o - NA * NC; row = A.c1 + r / ND; col = B.c2 + r % ND; }
                else if (o < NA * NC + NA * ND + NB * NC) { int r = o - NA * NC - NA * ND; row = A.c2 + r / NC; col = B.c1 + r % NC; }
                else { int r = o - NA * NC - NA * ND - NB * NC; row = A.c2 + r / ND; col = B.c2 + r % ND; }
                sD[o] = a.D[(int64_t)row * n + col];
            }
            const double *Dac = sD, *Dad = sD + NA * NC, *Dbc = Dad + NA * ND, *Dbd = Dbc + NB * NC;

            double gA[3] = {0.0, 0.0, 0.0}, gS[3] = {0.0, 0.0, 0.0}, gC[3] = {0.0, 0.0, 0.0};
            const double qk0 = a.pp[B.poff].q;
            // bra contraction of the chunk [cd0, cd0 + ncd) held in sX, sXc: lane ab
            // adds its weighted terms into gA, gS, gC
            auto bra_pass = [&](int cd0, int ncd, double a2) {
                        for (int r = 0; r < C::NABCH; ++r) {
                            const int ab = r * 64 + lane;
                            if (ab >= NAB) continue;
                            const int i = ab / NB, j = ab % NB;
                            int ax, ay, az, bx, by, bz;
                            cart_rt(LA, i, ax, ay, az);
                            cart_rt(LB, j, bx, by, bz);
                            double wv[CDCH];
#pragma unroll
                            for (int c = 0; c < CDCH; ++c) {
                                wv[c] = 0.0;
                                if (c < ncd) {
                                    const int kk = (cd0 + c) / ND, ll = (cd0 + c) % ND;
                                    wv[c] = -sdeg * (Dac[i * NC + kk] * Dbd[j * ND + ll] + Dad[i * ND + ll] * Dbc[j * NC + kk]);
                                }
                            }
                            const double *Ex = sEb, *Ey = sEb + C::EBD, *Ez = sEb + 2 * C::EBD;
                            const int ex_ = ax + bx, ey_ = ay + by, ez_ = az + bz;
                            const int ox = ax * C::EBI + bx * C::EBJ, oy = ay * C::EBI + by * C::EBJ,
                                      oz = az * C::EBI + bz * C::EBJ;
                            // One pass over the lane's Hermite box grown by one along
                            // every axis: each index t gets its weighted ket sum
                            //     z_t = sum_c w_c X_t(c)
                            // once, shared by the three d/dA terms (derivative
                            // coefficient along k times E along the other two) and the
                            // three (d/dA + d/dB) terms (E at t - 1_k).  E vanishes past
                            // the box, so indices beyond it along two axes carry no term
                            // and are skipped.  Walked as one flat loop of the class's
                            // largest grown box.
                            constexpr int UBM = box_max_grown(LA, LB);
                            const int mx = ex_ + 2, my = ey_ + 2, mz = ez_ + 2, nbox = mx * my * mz;
                            int tx = 0, ty = 0, tz = 0;
                            for (int st = 0; st < UBM; ++st) {
                                if (st < nbox && (tx > ex_) + (ty > ey_) + (tz > ez_) <= 1) {
                                    const double *xr = sX + herm_idx_rt(tx, ty, tz);
                                    double z = 0.0;
#pragma unroll
                                    for (int c = 0; c < CDCH; ++c) z += wv[c] * xr[c * NHX];
                                    const double e0 = Ex[ox + tx], e1 = Ey[oy + ty], e2 = Ez[oz + tz];
                                    const double d0 = dcoef(Ex, C::EBI, C::EBJ, ax, bx, tx, a2);
                                    const double d1 = dcoef(Ey, C::EBI, C::EBJ, ay, by, ty, a2);
                                    const double d2 = dcoef(Ez, C::EBI, C::EBJ, az, bz, tz, a2);
                                    gA[0] += d0 * e1 * e2 * z;
                                    gA[1] += e0 * d1 * e2 * z;
                                    gA[2] += e0 * e1 * d2 * z;
                                    if (tx > 0) gS[0] += Ex[ox + tx - 1] * e1 * e2 * z;
                                    if (ty > 0) gS[1] += e0 * Ey[oy + ty - 1] * e2 * z;
                                    if (tz > 0) gS[2] += e0 * e1 * Ez[oz + tz - 1] * z;
                                    if (tx <= ex_ && ty <= ey_ && tz <= ez_) {  // d/dC from Xc
                                        const int it = herm_idx_rt(tx, ty, tz);
                                        const double e = e0 * e1 * e2;
#pragma unroll
                                        for (int k = 0; k < 3; ++k) {
                                            double ac = 0.0;
#pragma unroll
                                            for (int c = 0; c < CDCH; ++c) ac += wv[c] * sXc[(k * CDCH + c) * NHC + it];
                                            gC[k] += e * ac;
                                        }
                                    }
                                }
                                if (++tz == mz) {
                                    tz = 0;
                                    if (++ty == my) {
                                        ty = 0;
                                        ++tx;
                                    }
                                }
                            }
                        }
            };
            for (int ip = 0; ip < A.np; ++ip) {
                const PrimPair pb = a.pp[A.poff + ip];
                if (pb.q * qk0 < a.tau_prim) break;
                if constexpr (KACC) {  // ket sums of this bra primitive pair start at zero
                    for (int o = lane; o < NCD * NHX; o += 64) sX[o] = 0.0;
                    for (int o = lane; o < 3 * CDCH * NHC; o += 64) sXc[o] = 0.0;
                }
                for (int kp = 0; kp < B.np; ++kp) {
                    const PrimPair pk = a.pp[B.poff + kp];
                    if (pb.q * pk.q < a.tau_prim) break;
                    const QuartetGeo geo = quartet_geo(pb, pk, a.om2);
                    wave_boys<L + 1>(geo, a.boys, sF, lane);
                    wave_hpoly<L + 1>(geo, sH, lane);
                    if (lane >= 8 && lane < 11) {
                        const int k = lane - 8;
                        const double pa = k == 0 ? pb.PA[0] : (k == 1 ? pb.PA[1] : pb.PA[2]);
                        const double pbb = k == 0 ? pb.PB[0] : (k == 1 ? pb.PB[1] : pb.PB[2]);
                        etab_lds<LA + 1, LB>(pa, pbb, pb.o2p, sEb + k * C::EBD);
                    } else if (lane >= 16 && lane < 19) {
                        const int k = lane - 16;
                        const double pa = k == 0 ? pk.PA[0] : (k == 1 ? pk.PA[1] : pk.PA[2]);
                        const double pbb = k == 0 ? pk.PB[0] : (k == 1 ? pk.PB[1] : pk.PB[2]);
                        etab_lds<LC + 1, LD>(pa, pbb, pk.o2p, sEk + k * C::EKD);
                    }
                    __syncthreads();
                    if constexpr (PLAN)
                        wave_r0h_plan<L + 1, double, L2 * L2, L2>(r0p, sF, sH, sR0, lane);
                    else
                        wave_r0h<L + 1>(sF, sH, sHerm, sR0, lane);
                    __syncthreads();
                    const double a2 = 2.0 * pb.a, c2 = 2.0 * pk.a;

                    for (int cd0 = 0; cd0 < NCD; cd0 += CDCH) {
                        const int ncd = (cd0 + CDCH < NCD) ? CDCH : NCD - cd0;
                        // ket coefficient lists of this chunk: for component cd and
                        // kq (0: E^{cd}, 1..3: its derivative along x, y, z) the
                        // coefficients (-1)^{|s|} Ed_s over the (extended) ket box and
                        // the R offsets of the box points, padded to KBM with zeros
                        for (int o = lane; o < 4 * ncd * C::KBM; o += 64) {
                            const int k = o % C::KBM, c = (o / C::KBM) % ncd, kq = o / (C::KBM * ncd);
                            const int kdir = kq - 1, cd = cd0 + c;
                            int cx, cy, cz, dx, dy, dz;
                            cart_rt(LC, cd / ND, cx, cy, cz);
                            cart_rt(LD, cd % ND, dx, dy, dz);
                            const int mx = cx + dx + 1 + (kdir == 0), my = cy + dy + 1 + (kdir == 1),
                                      mz = cz + dz + 1 + (kdir == 2);
                            double coef = 0.0;
                            int off = 0;
                            if (k < mx * my * mz) {
                                const int sx = k / (my * mz), sy = (k / mz) % my, sz = k % mz;
                                const double *Ex = sEk, *Ey = sEk + C::EKD, *Ez = sEk + 2 * C::EKD;
                                const double ex = kdir == 0 ? dcoef(Ex, C::EKI, C::EKJ, cx, dx, sx, c2)
                                                            : Ex[cx * C::EKI + dx * C::EKJ + sx];
                                const double ey = kdir == 1 ? dcoef(Ey, C::EKI, C::EKJ, cy, dy, sy, c2)
                                                            : Ey[cy * C::EKI + dy * C::EKJ + sy];
                                const double ez = kdir == 2 ? dcoef(Ez, C::EKI, C::EKJ, cz, dz, sz, c2)
                                                            : Ez[cz * C::EKI + dz * C::EKJ + sz];
                                coef = ((sx + sy + sz) & 1) ? -ex * ey * ez : ex * ey * ez;
                                off = (sx * L2 + sy) * L2 + sz;
                            }
                            sEc[(kq * CDCH + c) * C::KBM + k] = coef;
                            sEo[(kq * CDCH + c) * C::KBM + k] = off;
                        }
                        __syncthreads();
                        // ket-contracted intermediates of this chunk: one dot product
                        // of a coefficient list with R around t per output (the
                        // padding adds zeros times R_t, inside the table)
                        for (int o = lane; o < ncd * (NHX + 3 * NHC); o += 64) {
                            int c, t, kq;
                            if (o < ncd * NHX) { c = o / NHX; t = o % NHX; kq = 0; }
                            else { const int r = o - ncd * NHX; kq = 1 + r / (ncd * NHC); c = (r / NHC) % ncd; t = r % NHC; }
                            const int code = c_herm.tuv[t];
                            const int tb = ((code & 0xff) * L2 + ((code >> 8) & 0xff)) * L2 + (code >> 16);
                            const double *ec = sEc + (kq * CDCH + c) * C::KBM;
                            const int *eo = sEo + (kq * CDCH + c) * C::KBM;
                            double acc = 0.0;
#pragma unroll
                            for (int k = 0; k < C::KBM; ++k) acc += ec[k] * sR0[tb + eo[k]];
                            double &dst = kq == 0 ? sX[c * NHX + t] : sXc[((kq - 1) * CDCH + c) * NHC + t];
                            if constexpr (KACC) dst += acc; else dst = acc;
                        }
                        __syncthreads();

                        if constexpr (!KACC) {
                            bra_pass(cd0, ncd, a2);
                            __syncthreads();
                        }
                    }
                }
                if constexpr (KACC) {  // one bra contraction per bra primitive pair
                    bra_pass(0, NCD, 2.0 * pb.a);
                    __syncthreads();
                }
            }
            // wave sums (fixed butterfly), then one lane adds the four centres in order
            double v[9] = {gA[0], gA[1], gA[2], gS[0], gS[1], gS[2], gC[0], gC[1], gC[2]};
#pragma unroll
            for (int q = 0; q < 9; ++q)
                for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off);
            if (lane == 0) {
                for (int k = 0; k < 3; ++k) {
                    sG[3 * A.at1 + k] += v[k];
                    sG[3 * A.at2 + k] += v[3 + k] - v[k];
                    sG[3 * B.at1 + k] += v[6 + k];
                    sG[3 * B.at2 + k] += -v[3 + k] - v[6 + k];
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();
    for (int o = lane; o < na3; o += 64) g.partial[(int64_t)blockIdx.x * na3 + o] = sG[o];
}

template <int LA, int LB, int LC, int LD>
void launch_kg_t(const KGArgs &g, int blocks, hipStream_t st)
{
    if (blocks <= 0) return;
    const size_t shm = (size_t)3 * g.natom * sizeof(double);
    hipLaunchKernelGGL((kg_wave<LA, LB, LC, LD>), dim3((unsigned)blocks), dim3(64), shm, st, g);
}

template <int LA, int LB, int LC, int LD>
constexpr int kg_ranges_per_block()
{
    return KGCfg<LA, LB, LC, LD>::RANGE;
}

}  // namespace md

namespace md {

// ---------------------------------------------------------------------------
// Exchange gradient for the small classes: one lane per canonical quartet,
// every table in registers (the same sums as kg_wave, unrolled at compile
// time).  The 64 lanes of a wavefront stage their twelve centre terms in LDS
// and lanes owning (atom, axis) entries add them in lane order, so the
// per-workgroup partials are deterministic.
// ---------------------------------------------------------------------------
template <int LA, int LB, int LC, int LD>
__global__ __launch_bounds__(64) void kg_small(KGArgs g)
{
    constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
    constexpr int L = LA + LB + LC + LD, LAB = LA + LB;
    const KArgs &a = g.k;
    __shared__ double sT[64][13];  // 12 centre terms + valid flag per lane
    __shared__ int sAt[64][4];
    extern __shared__ double sG[];  // natom x 3
    const int lane = threadIdx.x;
    const int na3 = 3 * g.natom;
    for (int o = lane; o < na3; o += 64) sG[o] = 0.0;

    for (int64_t wbase = (int64_t)blockIdx.x * 64; wbase < a.nwork; wbase += (int64_t)gridDim.x * 64) {
        const int64_t w = wbase + lane;
        double v[12];
#pragma unroll
        for (int q = 0; q < 12; ++q) v[q] = 0.0;
        int at[4] = {0, 0, 0, 0};
        const bool valid = w < a.nwork;
        if (valid) {
            const int row = k_find_row(a.prefix, a.nrows, w);
            const int2 rw = a.rows[row];
            const CPair A = a.bra[rw.x], B = a.ket[rw.y + (int)(w - a.prefix[row])];
            at[0] = A.at1; at[1] = A.at2; at[2] = B.at1; at[3] = B.at2;
            double sdeg = 1.0;
            if (A.sh1 == A.sh2) sdeg *= 0.5;
            if (B.sh1 == B.sh2) sdeg *= 0.5;
            if (a.same && same_pair(A, B)) sdeg *= 0.5;
            const int n = a.ld;
            // weights W_{ab,cd} = -s (D_ac D_bd + D_ad D_bc)
            double W[NA * NB * NC * ND];
            static_for<0, NA * NB * NC * ND>([&](auto ec) {
                constexpr int e = decltype(ec)::value;
                constexpr int i = e / (NB * NC * ND), j = (e / (NC * ND)) % NB, k = (e / ND) % NC, l = e % ND;
                W[e] = -sdeg * (a.D[(int64_t)(A.c1 + i) * n + B.c1 + k] * a.D[(int64_t)(A.c2 + j) * n + B.c2 + l] +
                                a.D[(int64_t)(A.c1 + i) * n + B.c2 + l] * a.D[(int64_t)(A.c2 + j) * n + B.c1 + k]);
            });
            double gA[3] = {0, 0, 0}, gS[3] = {0, 0, 0}, gC[3] = {0, 0, 0};
            const double qk0 = a.pp[B.poff].q;
            for (int ip = 0; ip < A.np; ++ip) {
                const PrimPair pb = a.pp[A.poff + ip];
                if (pb.q * qk0 < a.tau_prim) break;
                Etab<LA + 1, LB> Ex, Ey, Ez;
                etab_build<LA + 1, LB>(pb.PA[0], pb.PB[0], pb.o2p, Ex);
                etab_build<LA + 1, LB>(pb.PA[1], pb.PB[1], pb.o2p, Ey);
                etab_build<LA + 1, LB>(pb.PA[2], pb.PB[2], pb.o2p, Ez);
                const double a2 = 2.0 * pb.a;
                for (int kp = 0; kp < B.np; ++kp) {
                    const PrimPair pk = a.pp[B.poff + kp];
                    if (pb.q * pk.q < a.tau_prim) break;
                    double Fs[L + 2], X, Y, Z;
                    quartet_fs<L + 1, double>(pb, pk, a.boys, Fs, X, Y, Z, a.om2);
                    double R[nherm(L + 1)];
                    r_build<L + 1, double>(Fs, X, Y, Z, R);
                    Etab<LC + 1, LD> Fx, Fy, Fz;
                    etab_build<LC + 1, LD>(pk.PA[0], pk.PB[0], pk.o2p, Fx);
                    etab_build<LC + 1, LD>(pk.PA[1], pk.PB[1], pk.o2p, Fy);
                    etab_build<LC + 1, LD>(pk.PA[2], pk.PB[2], pk.o2p, Fz);
                    const double c2 = 2.0 * pk.a;
                    static_for<0, NC * ND>([&](auto cdc) {
                        constexpr int cd = decltype(cdc)::value;
                        constexpr int c = cd / ND, d = cd % ND;
                        constexpr int cx = cart_x(LC, c), cy = cart_y(LC, c), cz = cart_z(LC, c);
                        constexpr int dx = cart_x(LD, d), dy = cart_y(LD, d), dz = cart_z(LD, d);
                        // X_t = sum_s (-1)^|s| E^{cd}_s R_{t+s}, t in H(LAB+1)
                        double Xt[nherm(LAB + 1)];
                        static_for<0, nherm(LAB + 1)>([&](auto pc) {
                            constexpr int P = decltype(pc)::value;
                            constexpr int tp = herm_t(P), up = herm_u(P), vp = herm_v(P);
                            double s = 0.0;
                            static_for<0, cx + dx + 1>([&](auto sxc) {
                                constexpr int sx = decltype(sxc)::value;
                                static_for<0, cy + dy + 1>([&](auto syc) {
                                    constexpr int sy = decltype(syc)::value;
                                    static_for<0, cz + dz + 1>([&](auto szc) {
                                        constexpr int sz = decltype(szc)::value;
                                        constexpr double sg = ((sx + sy + sz) & 1) ? -1.0 : 1.0;
                                        s += sg * Fx.e[cx][dx][sx] * Fy.e[cy][dy][sy] * Fz.e[cz][dz][sz] *
                                             R[herm_idx(tp + sx, up + sy, vp + sz)];
                                    });
                                });
                            });
                            Xt[P] = s;
                        });
                        // Xc^k_t = sum_s (-1)^|s| Ed^{C,k}_s R_{t+s}, t in H(LAB)
                        double Xc[3][nherm(LAB)];
                        static_for<0, 3>([&](auto kc) {
                            constexpr int k = decltype(kc)::value;
                            static_for<0, nherm(LAB)>([&](auto pc) {
                                constexpr int P = decltype(pc)::value;
                                constexpr int tp = herm_t(P), up = herm_u(P), vp = herm_v(P);
                                double s = 0.0;
                                static_for<0, cx + dx + 1 + (k == 0)>([&](auto sxc) {
                                    constexpr int sx = decltype(sxc)::value;
                                    double ex;
                                    if constexpr (k == 0) {
                                        ex = c2 * Fx.e[cx + 1][dx][sx];
                                        if constexpr (cx > 0 && sx <= cx - 1 + dx) ex -= (double)cx * Fx.e[cx - 1][dx][sx];
                                    } else {
                                        ex = Fx.e[cx][dx][sx];
                                    }
                                    static_for<0, cy + dy + 1 + (k == 1)>([&](auto syc) {
                                        constexpr int sy = decltype(syc)::value;
                                        double ey;
                                        if constexpr (k == 1) {
                                            ey = c2 * Fy.e[cy + 1][dy][sy];
                                            if constexpr (cy > 0 && sy <= cy - 1 + dy) ey -= (double)cy * Fy.e[cy - 1][dy][sy];
                                        } else {
                                            ey = Fy.e[cy][dy][sy];
                                        }
                                        static_for<0, cz + dz + 1 + (k == 2)>([&](auto szc) {
                                            constexpr int sz = decltype(szc)::value;
                                            double ez;
                                            if constexpr (k == 2) {
                                                ez = c2 * Fz.e[cz + 1][dz][sz];
                                                if constexpr (cz > 0 && sz <= cz - 1 + dz) ez -= (double)cz * Fz.e[cz - 1][dz][sz];
                                            } else {
                                                ez = Fz.e[cz][dz][sz];
                                            }
                                            constexpr double sg = ((sx + sy + sz) & 1) ? -1.0 : 1.0;
                                            s += sg * ex * ey * ez * R[herm_idx(tp + sx, up + sy, vp + sz)];
                                        });
                                    });
                                });
                                Xc[k][P] = s;
                            });
                        });
                        // bra side with the weights
                        static_for<0, NA * NB>([&](auto abc) {
                            constexpr int ab = decltype(abc)::value;
                            constexpr int i = ab / NB, j = ab % NB;
                            constexpr int ax = cart_x(LA, i), ay = cart_y(LA, i), az = cart_z(LA, i);
                            constexpr int bx = cart_x(LB, j), by = cart_y(LB, j), bz = cart_z(LB, j);
                            const double w = W[ab * (NC * ND) + cd];
                            // dA_k: coefficient boxes extended along k
                            static_for<0, 3>([&](auto kc) {
                                constexpr int k = decltype(kc)::value;
                                double s = 0.0;
                                static_for<0, ax + bx + 1 + (k == 0)>([&](auto txc) {
                                    constexpr int tx = decltype(txc)::value;
                                    double fx;
                                    if constexpr (k == 0) {
                                        fx = a2 * Ex.e[ax + 1][bx][tx];
                                        if constexpr (ax > 0 && tx <= ax - 1 + bx) fx -= (double)ax * Ex.e[ax - 1][bx][tx];
                                    } else {
                                        fx = Ex.e[ax][bx][tx];
                                    }
                                    static_for<0, ay + by + 1 + (k == 1)>([&](auto tyc) {
                                        constexpr int ty = decltype(tyc)::value;
                                        double fy;
                                        if constexpr (k == 1) {
                                            fy = a2 * Ey.e[ay + 1][by][ty];
                                            if constexpr (ay > 0 && ty <= ay - 1 + by) fy -= (double)ay * Ey.e[ay - 1][by][ty];
                                        } else {
                                            fy = Ey.e[ay][by][ty];
                                        }
                                        static_for<0, az + bz + 1 + (k == 2)>([&](auto tzc) {
                                            constexpr int tz = decltype(tzc)::value;
                                            double fz;
                                            if constexpr (k == 2) {
                                                fz = a2 * Ez.e[az + 1][bz][tz];
                                                if constexpr (az > 0 && tz <= az - 1 + bz) fz -= (double)az * Ez.e[az - 1][bz][tz];
                                            } else {
                                                fz = Ez.e[az][bz][tz];
                                            }
                                            s += fx * fy * fz * Xt[herm_idx(tx, ty, tz)];
                                        });
                                    });
                                });
                                gA[k] += w * s;
                            });
                            // (dA + dB) by the index shift, dC from Xc
                            static_for<0, ax + bx + 1>([&](auto txc) {
                                constexpr int tx = decltype(txc)::value;
                                static_for<0, ay + by + 1>([&](auto tyc) {
                                    constexpr int ty = decltype(tyc)::value;
                                    static_for<0, az + bz + 1>([&](auto tzc) {
                                        constexpr int tz = decltype(tzc)::value;
                                        const double e = w * Ex.e[ax][bx][tx] * Ey.e[ay][by][ty] * Ez.e[az][bz][tz];
                                        gS[0] += e * Xt[herm_idx(tx + 1, ty, tz)];
                                        gS[1] += e * Xt[herm_idx(tx, ty + 1, tz)];
                                        gS[2] += e * Xt[herm_idx(tx, ty, tz + 1)];
                                        gC[0] += e * Xc[0][herm_idx(tx, ty, tz)];
                                        gC[1] += e * Xc[1][herm_idx(tx, ty, tz)];
                                        gC[2] += e * Xc[2][herm_idx(tx, ty, tz)];
                                    });
                                });
                            });
                        });
                    });
                }
            }
            for (int k = 0; k < 3; ++k) {
                v[k] = gA[k];
                v[3 + k] = gS[k] - gA[k];
                v[6 + k] = gC[k];
                v[9 + k] = -gS[k] - gC[k];
            }
        }
        // stage and add in lane order (deterministic)
#pragma unroll
        for (int q = 0; q < 12; ++q) sT[lane][q] = v[q];
        sT[lane][12] = valid ? 1.0 : 0.0;
        for (int c = 0; c < 4; ++c) sAt[lane][c] = at[c];
        __syncthreads();
        for (int o = lane; o < na3; o += 64) {
            const int atom = o / 3, k = o % 3;
            double acc = 0.0;
            for (int l = 0; l < 64; ++l) {
                if (sT[l][12] == 0.0) continue;
                for (int c = 0; c < 4; ++c)
                    if (sAt[l][c] == atom) acc += sT[l][3 * c + k];
            }
            sG[o] += acc;
        }
        __syncthreads();
    }
    for (int o = lane; o < na3; o += 64) g.partial[(int64_t)blockIdx.x * na3 + o] = sG[o];
}

template <int LA, int LB, int LC, int LD>
void launch_kg_small_t(const KGArgs &g, int blocks, hipStream_t st)
{
    if (blocks <= 0) return;
    const size_t shm = (size_t)3 * g.natom * sizeof(double);
    hipLaunchKernelGGL((kg_small<LA, LB, LC, LD>), dim3((unsigned)blocks), dim3(64), shm, st, g);
}

}  // namespace md

namespace md {

template <int LA, int LB, int LC, int LD>
constexpr bool kg_use_small()
{
    return kg_small_class(LA, LB, LC, LD);
}

template <int LA, int LB, int LC, int LD>
void launch_kg_any(const KGArgs &g, int blocks, hipStream_t st)
{
    if constexpr (kg_use_small<LA, LB, LC, LD>())
        launch_kg_small_t<LA, LB, LC, LD>(g, blocks, st);
    else
        launch_kg_t<LA, LB, LC, LD>(g, blocks, st);
}

}  // namespace md
