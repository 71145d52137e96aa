// setup.hip -- Schwarz factors (eq. cauchy_schwarz_bound), density and
// result basis transforms, and small utility kernels.
#include "kern_args.hpp"
#include "launch.hpp"
#include "md_device.hpp"
#include "wave_r.hpp"

namespace md {

// Real solid harmonics as combinations of x^l-normalised Cartesian
// primitives, rows m = -l..l (p kept as x, y, z):
//   d: sqrt3 xy, sqrt3 yz, z^2 - (x^2+y^2)/2, sqrt3 xz, sqrt3/2 (x^2 - y^2)
//   f: sqrt(5/8)(3x^2y - y^3), sqrt15 xyz, sqrt(3/8) y(4z^2 - x^2 - y^2),
//      z^3 - 3/2 z(x^2+y^2), sqrt(3/8) x(4z^2 - x^2 - y^2),
//      sqrt15/2 z(x^2 - y^2), sqrt(5/8)(x^3 - 3xy^2)
struct SphTables {
    double v[110];
    int off[4];
    constexpr SphTables() : v(), off{0, 1, 10, 40}
    {
        v[0] = 1.0;
        for (int i = 0; i < 3; ++i) v[1 + i * 3 + i] = 1.0;
        const double s3 = 1.7320508075688772935;
        double *d = v + 10;  // 5 x 6: xx xy xz yy yz zz
        d[0 * 6 + 1] = s3;
        d[1 * 6 + 4] = s3;
        d[2 * 6 + 0] = -0.5; d[2 * 6 + 3] = -0.5; d[2 * 6 + 5] = 1.0;
        d[3 * 6 + 2] = s3;
        d[4 * 6 + 0] = 0.5 * s3; d[4 * 6 + 3] = -0.5 * s3;
        const double a58 = 0.79056941504209483300;  // sqrt(5/8)
        const double a38 = 0.61237243569579452455;  // sqrt(3/8)
        const double s15 = 3.8729833462074168852;
        double *f = v + 40;  // 7 x 10: xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz
        f[0 * 10 + 1] = 3.0 * a58; f[0 * 10 + 6] = -a58;
        f[1 * 10 + 4] = s15;
        f[2 * 10 + 8] = 4.0 * a38; f[2 * 10 + 1] = -a38; f[2 * 10 + 6] = -a38;
        f[3 * 10 + 9] = 1.0; f[3 * 10 + 2] = -1.5; f[3 * 10 + 7] = -1.5;
        f[4 * 10 + 5] = 4.0 * a38; f[4 * 10 + 0] = -a38; f[4 * 10 + 3] = -a38;
        f[5 * 10 + 2] = 0.5 * s15; f[5 * 10 + 7] = -0.5 * s15;
        f[6 * 10 + 0] = a58; f[6 * 10 + 3] = -3.0 * a58;
    }
};
__constant__ const SphTables c_sph{};

// P_cart = T^T P_sym T with P_sym = (P + P^T)/2 (identity T when Cartesian)
__global__ void p_to_cart(const double *__restrict__ P, int nbf, double *__restrict__ Pc, int nc,
                          ShellMap m, int spherical)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nc * nc) return;
    const int i = (int)(idx / nc), j = (int)(idx % nc);
    if (!spherical) {
        Pc[idx] = 0.5 * (P[(int64_t)i * nbf + j] + P[(int64_t)j * nbf + i]);
        return;
    }
    const int si = m.shell_of_cart[i], sj = m.shell_of_cart[j];
    const int li = m.l[si], lj = m.l[sj];
    const int ci = i - m.cart_off[si], cj = j - m.cart_off[sj];
    const int oi = m.sph_off[si], oj = m.sph_off[sj];
    const double *Ti = c_sph.v + c_sph.off[li];
    const double *Tj = c_sph.v + c_sph.off[lj];
    const int nci = ncart(li), ncj = ncart(lj);
    double acc = 0.0;
    for (int a = 0; a < 2 * li + 1; ++a) {
        const double ta = Ti[a * nci + ci];
        if (ta == 0.0) continue;
        for (int b = 0; b < 2 * lj + 1; ++b) {
            const double tb = Tj[b * ncj + cj];
            if (tb == 0.0) continue;
            acc += ta * tb * 0.5 * (P[(int64_t)(oi + a) * nbf + oj + b] + P[(int64_t)(oj + b) * nbf + oi + a]);
        }
    }
    Pc[idx] = acc;
}

// Out = T (Acc + Acc^T) T^T (Out = Acc + Acc^T when Cartesian)
__global__ void acc_to_out(const double *__restrict__ Acc, int nc, double *__restrict__ Out, int nbf,
                           ShellMap m, int spherical)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nbf * nbf) return;
    const int r = (int)(idx / nbf), c = (int)(idx % nbf);
    if (!spherical) {
        Out[idx] = Acc[(int64_t)r * nc + c] + Acc[(int64_t)c * nc + r];
        return;
    }
    const int sr = m.shell_of_sph[r], sc = m.shell_of_sph[c];
    const int lr = m.l[sr], lc = m.l[sc];
    const int mr = r - m.sph_off[sr], mc = c - m.sph_off[sc];
    const int orr = m.cart_off[sr], oc = m.cart_off[sc];
    const int nr = ncart(lr), ncc = ncart(lc);
    const double *Tr = c_sph.v + c_sph.off[lr] + mr * nr;
    const double *Tc = c_sph.v + c_sph.off[lc] + mc * ncc;
    double acc = 0.0;
    for (int a = 0; a < nr; ++a) {
        const double ta = Tr[a];
        if (ta == 0.0) continue;
        for (int b = 0; b < ncc; ++b) {
            const double tb = Tc[b];
            if (tb == 0.0) continue;
            acc += ta * tb * (Acc[(int64_t)(orr + a) * nc + oc + b] + Acc[(int64_t)(oc + b) * nc + orr + a]);
        }
    }
    Out[idx] = acc;
}

__global__ void fill_zero(double *__restrict__ x, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = 0.0;
}

// Schwarz factors: one wavefront per contracted pair.  For every primitive
// pair q = sqrt(max_c |(ij|ij)_c|) is written into PrimPair::q; for the
// contracted pair Q = sqrt(max_c |(ab|ab)_c|) over all primitive quartets.
template <int LA, int LB>
__global__ __launch_bounds__(64) void schwarz_wave(const CPair *__restrict__ cp, int ncp,
                                                   PrimPair *__restrict__ pp, double *__restrict__ Q,
                                                   const double *__restrict__ boys)
{
    constexpr int NA = ncart(LA), NB = ncart(LB), NAB = NA * NB, LAB = LA + LB;
    constexpr int L = 2 * LAB, L1 = L + 1;
    constexpr int EBD = (LA + 1) * (LB + 1) * (LAB + 1);
    __shared__ double sR0[L1 * L1 * L1];
    __shared__ double sF[L + 1];
    __shared__ double sPow[3 * (L + 1)];
    __shared__ double sEb[3 * EBD];
    __shared__ double sEk[3 * EBD];
    const int lane = threadIdx.x;
    int comp[2][6];
    bool own[2];
    for (int r = 0; r < 2; ++r) {
        const int ab = lane + 64 * r;
        own[r] = ab < NAB;
        int ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
        if (own[r]) {
            cart_rt(LA, ab / NB, ax, ay, az);
            cart_rt(LB, ab % NB, bx, by, bz);
        }
        comp[r][0] = ax; comp[r][1] = ay; comp[r][2] = az;
        comp[r][3] = bx; comp[r][4] = by; comp[r][5] = bz;
    }
    for (int c = blockIdx.x; c < ncp; c += gridDim.x) {
        const CPair A = cp[c];
        double dsum[2] = {0.0, 0.0};
        for (int ip = 0; ip < A.np; ++ip) {
            const PrimPair pb = pp[A.poff + ip];
            for (int kp = 0; kp < A.np; ++kp) {
                const PrimPair pk = pp[A.poff + kp];
                const QuartetGeo g = quartet_geo(pb, pk, 0.0);  // screening bounds of 1/r
                wave_boys<L>(g, boys, sF, lane);
                wave_powers<L>(g, sPow, lane);
                if (lane >= 61) {
                    const int ax = lane - 61;
                    const double pa = ax == 0 ? pb.PA[0] : (ax == 1 ? pb.PA[1] : pb.PA[2]);
                    const double pbb = ax == 0 ? pb.PB[0] : (ax == 1 ? pb.PB[1] : pb.PB[2]);
                    etab_reg_store<LA, LB>(pa, pbb, pb.o2p, sEb + ax * EBD);
                } else if (lane >= 58) {
                    const int ax = lane - 58;
                    const double pa = ax == 0 ? pk.PA[0] : (ax == 1 ? pk.PA[1] : pk.PA[2]);
                    const double pbb = ax == 0 ? pk.PB[0] : (ax == 1 ? pk.PB[1] : pk.PB[2]);
                    etab_reg_store<LA, LB>(pa, pbb, pk.o2p, sEk + ax * EBD);
                }
                __syncthreads();
                wave_r0<L>(sF, sPow, sR0, lane);
                __syncthreads();
                double pd = 0.0;
                for (int r = 0; r < 2; ++r) {
                    if (!own[r]) continue;
                    const int ax = comp[r][0], ay = comp[r][1], az = comp[r][2];
                    const int bx = comp[r][3], by = comp[r][4], bz = comp[r][5];
                    const double *Ebx = sEb + (ax * (LB + 1) + bx) * (LAB + 1);
                    const double *Eby = sEb + EBD + (ay * (LB + 1) + by) * (LAB + 1);
                    const double *Ebz = sEb + 2 * EBD + (az * (LB + 1) + bz) * (LAB + 1);
                    const double *Ekx = sEk + (ax * (LB + 1) + bx) * (LAB + 1);
                    const double *Eky = sEk + EBD + (ay * (LB + 1) + by) * (LAB + 1);
                    const double *Ekz = sEk + 2 * EBD + (az * (LB + 1) + bz) * (LAB + 1);
                    double v = 0.0;
                    for (int tx = 0; tx <= ax + bx; ++tx)
                        for (int ty = 0; ty <= ay + by; ++ty)
                            for (int tz = 0; tz <= az + bz; ++tz) {
                                const double e = Ebx[tx] * Eby[ty] * Ebz[tz];
                                double s = 0.0;
                                for (int sx = 0; sx <= ax + bx; ++sx)
                                    for (int sy = 0; sy <= ay + by; ++sy)
                                        for (int sz = 0; sz <= az + bz; ++sz) {
                                            const double sg = ((sx + sy + sz) & 1) ? -1.0 : 1.0;
                                            s += sg * Ekx[sx] * Eky[sy] * Ekz[sz] *
                                                 sR0[((tx + sx) * L1 + ty + sy) * L1 + tz + sz];
                                        }
                                v += e * s;
                            }
                    dsum[r] += v;
                    pd = fmax(pd, fabs(v));
                }
                if (ip == kp) {
                    for (int off = 32; off > 0; off >>= 1) pd = fmax(pd, __shfl_xor(pd, off));
                    if (lane == 0) pp[A.poff + ip].q = sqrt(pd);
                }
                __syncthreads();
            }
        }
        double m = fmax(fabs(dsum[0]), fabs(dsum[1]));
        for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
        if (lane == 0) Q[c] = sqrt(m);
        __syncthreads();
    }
}

void launch_schwarz(int la, int lb, const CPair *cp, int ncp, PrimPair *pp, double *Q,
                    const double *boys, hipStream_t st)
{
    if (ncp <= 0) return;
    const int blocks = ncp < 8192 ? ncp : 8192;
#define MD_SW(A_, B_)                                                                           \
    if (la == A_ && lb == B_) {                                                                \
        hipLaunchKernelGGL((schwarz_wave<A_, B_>), dim3(blocks), dim3(64), 0, st, cp, ncp, pp, Q, boys); \
        return;                                                                                \
    }
    MD_SW(0, 0) MD_SW(1, 0) MD_SW(1, 1) MD_SW(2, 0) MD_SW(2, 1) MD_SW(2, 2) MD_SW(3, 0) MD_SW(3, 1)
    MD_SW(3, 2) MD_SW(3, 3)
#undef MD_SW
}

void launch_p_to_cart(const double *P, int nbf, double *Pc, int nc, const ShellMap &m, int sph,
                      hipStream_t st)
{
    const int64_t n = (int64_t)nc * nc;
    hipLaunchKernelGGL(p_to_cart, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, nbf, Pc, nc, m, sph);
}

void launch_acc_to_out(const double *Acc, int nc, double *Out, int nbf, const ShellMap &m, int sph,
                       hipStream_t st)
{
    const int64_t n = (int64_t)nbf * nbf;
    hipLaunchKernelGGL(acc_to_out, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Acc, nc, Out, nbf, m, sph);
}

// Density bounds of the mixed-precision rule: Pm[s1][s2] = max |P_cart| over
// the (s1, s2) shell block, one thread per block.
__global__ void shell_pair_pmax(const double *__restrict__ Pc, int nc, const int32_t *__restrict__ l,
                                const int32_t *__restrict__ coff, int nsh, double *__restrict__ Pm)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nsh * nsh) return;
    const int s1 = (int)(idx / nsh), s2 = (int)(idx % nsh);
    const int n1 = ncart(l[s1]), n2 = ncart(l[s2]), o1 = coff[s1], o2 = coff[s2];
    double m = 0.0;
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j) m = fmax(m, fabs(Pc[(int64_t)(o1 + i) * nc + o2 + j]));
    Pm[idx] = m;
}

// QD[k] = Q_k max|D| over the shell block of contracted pair k (J-engine kets).
__global__ void pair_qd(const CPair *__restrict__ cp, const double *__restrict__ Q, int n,
                        const double *__restrict__ Pm, int nsh, double *__restrict__ QD)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const CPair c = cp[k];
    QD[k] = Q[k] * Pm[(int64_t)c.sh1 * nsh + c.sh2];
}

void launch_density_bounds(const double *Pc, int nc, const int32_t *l, const int32_t *coff, int nsh,
                           double *Pm, const CPair *cp, const double *Q, int ncp, double *QD, hipStream_t st)
{
    const int64_t n = (int64_t)nsh * nsh;
    hipLaunchKernelGGL(shell_pair_pmax, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Pc, nc, l, coff, nsh, Pm);
    if (ncp > 0)
        hipLaunchKernelGGL(pair_qd, dim3((unsigned)((ncp + 255) / 256)), dim3(256), 0, st, cp, Q, ncp, Pm, nsh, QD);
}

void launch_fill_zero(double *x, int64_t n, hipStream_t st)
{
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_zero, dim3((unsigned)blocks), dim3(256), 0, st, x, n);
}

}  // namespace md
