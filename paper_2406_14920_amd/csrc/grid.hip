// grid.hip -- the electron density and its gradient on grid points (eqs.
// xc_density_0, xc_density_1) and the exchange-correlation matrix sums over
// grid points (eqs. xc_grid_sum_0, xc_grid_sum_1), the grid-based step of the
// local exchange-correlation integrals (eq. xc_integral_definition).
//
// A contracted pair's product of basis functions at r factors into a
// polynomial of the two centres' offsets and a primitive sum:
//     a(r) b(r) = xa^i xb^j ya^k yb^l za^m zb^n * g(r),
//     g(r) = sum_k K_k exp(-p_k |r - P_k|^2)      (eq. pair_definition),
// and its derivative along x is (eq. pair_derivative)
//     d/dx = (i xa^{i-1} xb^j + j xa^i xb^{j-1}) (...) g + xa^i xb^j (...) dg/dx,
//     dg/dx = sum_k K_k (-2 p_k)(x - P_kx) exp(-p_k |r - P_k|^2).
// A primitive with p |r - P|^2 > 100 is dropped (exp(-100) ~ 4e-44, the
// paper's cut-off value).  Every contracted pair has a bounding sphere that
// holds all points where any of its primitives survives, every block of 64
// consecutive grid points a bounding sphere of its points; a pair and a block
// whose spheres do not meet are skipped as a whole (the paper's atom groups
// and grid boxes, with the pair and the wavefront as the units).
//
// Density: one lane per grid point, the contracted pairs of a class walked in
// order (wave-uniform, so pair data and density blocks arrive through scalar
// loads), sums added into rho[g] class by class: deterministic.
// Matrix: one wavefront per contracted pair, the lanes over the points of
// each nearby block, NA*NB sums per lane reduced across the wavefront in a
// fixed order, one triangle of the accumulator written (V = Acc + Acc^T).
#include "grid.hpp"
#include "kern_args.hpp"
#include "launch.hpp"
#include "md_device.hpp"

namespace md {

// block spheres: centre = mean of the block's points, radius = farthest point
__global__ __launch_bounds__(64) void grid_blocks(const double *__restrict__ pts, int64_t npts,
                                                  double4 *__restrict__ bsph)
{
    const int lane = threadIdx.x;
    const int64_t g = (int64_t)blockIdx.x * 64 + lane;
    const bool valid = g < npts;
    const int64_t gc = valid ? g : (int64_t)blockIdx.x * 64;
    const double x = pts[3 * gc], y = pts[3 * gc + 1], z = pts[3 * gc + 2];
    double sx = valid ? x : 0.0, sy = valid ? y : 0.0, sz = valid ? z : 0.0, n = valid ? 1.0 : 0.0;
    for (int off = 32; off > 0; off >>= 1) {
        sx += __shfl_xor(sx, off);
        sy += __shfl_xor(sy, off);
        sz += __shfl_xor(sz, off);
        n += __shfl_xor(n, off);
    }
    const double cx = sx / n, cy = sy / n, cz = sz / n;
    double r2 = valid ? (x - cx) * (x - cx) + (y - cy) * (y - cy) + (z - cz) * (z - cz) : 0.0;
    for (int off = 32; off > 0; off >>= 1) r2 = fmax(r2, __shfl_xor(r2, off));
    if (lane == 0) bsph[blockIdx.x] = make_double4(cx, cy, cz, sqrt(r2));
}

__device__ __forceinline__ bool spheres_meet(const double4 &a, const double4 &b)
{
    const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z, s = a.w + b.w;
    return dx * dx + dy * dy + dz * dz <= s * s;
}

// g(r) and its gradient for one contracted pair at one point
template <bool GRAD>
__device__ __forceinline__ void pair_gauss(const PrimPair *__restrict__ pp, const CPair &A, double x, double y,
                                           double z, double &g, double &gx, double &gy, double &gz)
{
    g = gx = gy = gz = 0.0;
    for (int k = 0; k < A.np; ++k) {
        const PrimPair &q = pp[A.poff + k];
        const double dx = x - q.P[0], dy = y - q.P[1], dz = z - q.P[2];
        const double t = q.p * (dx * dx + dy * dy + dz * dz);
        if (t > kGridCut) continue;
        const double v = q.K * exp(-t);
        g += v;
        if constexpr (GRAD) {
            const double m = -2.0 * q.p * v;
            gx += m * dx;
            gy += m * dy;
            gz += m * dz;
        }
    }
}

// powers u^0 .. u^N
template <int N>
__device__ __forceinline__ void powers(double u, double *o)
{
    o[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= N; ++k) o[k] = o[k - 1] * u;
}

// one Cartesian component pair (a, b): value of the polynomial and its three
// derivatives, from the per-axis powers of the offsets to A and B
template <int LA, int LB, int IA, int JB, bool GRAD>
__device__ __forceinline__ void poly_ab(const double (&pa)[3][LA + 1], const double (&pb)[3][LB + 1], double &v,
                                        double &vx, double &vy, double &vz)
{
    constexpr int ax = cart_x(LA, IA), ay = cart_y(LA, IA), az = cart_z(LA, IA);
    constexpr int bx = cart_x(LB, JB), by = cart_y(LB, JB), bz = cart_z(LB, JB);
    const double X = pa[0][ax] * pb[0][bx], Y = pa[1][ay] * pb[1][by], Z = pa[2][az] * pb[2][bz];
    v = X * Y * Z;
    if constexpr (GRAD) {
        double dX = 0.0, dY = 0.0, dZ = 0.0;
        if constexpr (ax > 0) dX += ax * pa[0][ax - 1] * pb[0][bx];
        if constexpr (bx > 0) dX += bx * pa[0][ax] * pb[0][bx - 1];
        if constexpr (ay > 0) dY += ay * pa[1][ay - 1] * pb[1][by];
        if constexpr (by > 0) dY += by * pa[1][ay] * pb[1][by - 1];
        if constexpr (az > 0) dZ += az * pa[2][az - 1] * pb[2][bz];
        if constexpr (bz > 0) dZ += bz * pa[2][az] * pb[2][bz - 1];
        vx = dX * Y * Z;
        vy = X * dY * Z;
        vz = X * Y * dZ;
    } else {
        vx = vy = vz = 0.0;
    }
}

template <int LA, int LB, bool GRAD>
__global__ __launch_bounds__(64) void grid_rho(const CPair *__restrict__ cp, int ncp, const PrimPair *__restrict__ pp,
                                               const double4 *__restrict__ psph, const double *__restrict__ xyz,
                                               const double *__restrict__ D, int ld, const double *__restrict__ pts,
                                               int64_t npts, const double4 *__restrict__ bsph,
                                               double *__restrict__ rho, double *__restrict__ grad)
{
    constexpr int NA = ncart(LA), NB = ncart(LB);
    const int64_t g = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const bool valid = g < npts;
    const int64_t gc = valid ? g : (int64_t)blockIdx.x * 64;
    const double x = pts[3 * gc], y = pts[3 * gc + 1], z = pts[3 * gc + 2];
    const double4 bs = bsph[blockIdx.x];
    double acc = 0.0, ax_ = 0.0, ay_ = 0.0, az_ = 0.0;
    for (int c = 0; c < ncp; ++c) {
        if (!spheres_meet(psph[c], bs)) continue;  // uniform over the wavefront
        const CPair A = cp[c];
        double e, ex, ey, ez;
        pair_gauss<GRAD>(pp, A, x, y, z, e, ex, ey, ez);
        double pa[3][LA + 1], pb[3][LB + 1];
        powers<LA>(x - xyz[3 * A.at1], pa[0]);
        powers<LA>(y - xyz[3 * A.at1 + 1], pa[1]);
        powers<LA>(z - xyz[3 * A.at1 + 2], pa[2]);
        powers<LB>(x - xyz[3 * A.at2], pb[0]);
        powers<LB>(y - xyz[3 * A.at2 + 1], pb[1]);
        powers<LB>(z - xyz[3 * A.at2 + 2], pb[2]);
        const double f = (A.sh1 == A.sh2) ? 1.0 : 2.0;
        double s = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
        static_for<0, NA * NB>([&](auto abc) {
            constexpr int ab = decltype(abc)::value;
            const double d = D[(int64_t)(A.c1 + ab / NB) * ld + A.c2 + ab % NB];
            double v, vx, vy, vz;
            poly_ab<LA, LB, ab / NB, ab % NB, GRAD>(pa, pb, v, vx, vy, vz);
            s += d * v;
            if constexpr (GRAD) {
                sx += d * vx;
                sy += d * vy;
                sz += d * vz;
            }
        });
        acc += f * s * e;
        if constexpr (GRAD) {
            ax_ += f * (sx * e + s * ex);
            ay_ += f * (sy * e + s * ey);
            az_ += f * (sz * e + s * ez);
        }
    }
    if (valid) {
        rho[g] += acc;
        if constexpr (GRAD) {
            grad[3 * g] += ax_;
            grad[3 * g + 1] += ay_;
            grad[3 * g + 2] += az_;
        }
    }
}

template <int LA, int LB, bool GRAD>
__global__ __launch_bounds__(64) void grid_vmat(const CPair *__restrict__ cp, int ncp, const PrimPair *__restrict__ pp,
                                                const double4 *__restrict__ psph, const double *__restrict__ xyz,
                                                const double *__restrict__ pts, int64_t npts, int nblk,
                                                const double4 *__restrict__ bsph, const double *__restrict__ v0,
                                                const double *__restrict__ v1, double *__restrict__ Vacc, int ld)
{
    constexpr int NA = ncart(LA), NB = ncart(LB), NAB = NA * NB;
    const int c = blockIdx.x;
    if (c >= ncp) return;
    const int lane = threadIdx.x;
    const CPair A = cp[c];
    const double4 ps = psph[c];
    const double Ax = xyz[3 * A.at1], Ay = xyz[3 * A.at1 + 1], Az = xyz[3 * A.at1 + 2];
    const double Bx = xyz[3 * A.at2], By = xyz[3 * A.at2 + 1], Bz = xyz[3 * A.at2 + 2];
    double acc[NAB];
#pragma unroll
    for (int i = 0; i < NAB; ++i) acc[i] = 0.0;
    for (int b = 0; b < nblk; ++b) {
        if (!spheres_meet(ps, bsph[b])) continue;  // uniform over the wavefront
        const int64_t g = (int64_t)b * 64 + lane;
        if (g >= npts) continue;  // no cross-lane work inside the loop
        const double x = pts[3 * g], y = pts[3 * g + 1], z = pts[3 * g + 2];
        double e, ex, ey, ez;
        pair_gauss<GRAD>(pp, A, x, y, z, e, ex, ey, ez);
        if (e == 0.0 && (!GRAD || (ex == 0.0 && ey == 0.0 && ez == 0.0))) continue;
        const double w0 = v0[g];
        double w1x = 0.0, w1y = 0.0, w1z = 0.0;
        if constexpr (GRAD) {
            w1x = v1[3 * g];
            w1y = v1[3 * g + 1];
            w1z = v1[3 * g + 2];
        }
        // weights of the polynomial and of its three derivatives
        const double cv = w0 * e + w1x * ex + w1y * ey + w1z * ez;
        const double cx = w1x * e, cy = w1y * e, cz = w1z * e;
        double pa[3][LA + 1], pb[3][LB + 1];
        powers<LA>(x - Ax, pa[0]);
        powers<LA>(y - Ay, pa[1]);
        powers<LA>(z - Az, pa[2]);
        powers<LB>(x - Bx, pb[0]);
        powers<LB>(y - By, pb[1]);
        powers<LB>(z - Bz, pb[2]);
        static_for<0, NAB>([&](auto abc) {
            constexpr int ab = decltype(abc)::value;
            double v, vx, vy, vz;
            poly_ab<LA, LB, ab / NB, ab % NB, GRAD>(pa, pb, v, vx, vy, vz);
            if constexpr (GRAD)
                acc[ab] += cv * v + cx * vx + cy * vy + cz * vz;
            else
                acc[ab] += cv * v;
        });
    }
    const double f = (A.sh1 == A.sh2) ? 0.5 : 1.0;
#pragma unroll
    for (int i = 0; i < NAB; ++i) {
        double v = acc[i];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) Vacc[(int64_t)(A.c1 + i / NB) * ld + A.c2 + i % NB] = f * v;
    }
}

void launch_grid_blocks(const double *pts, int64_t npts, double4 *bsph, hipStream_t st)
{
    if (npts <= 0) return;
    hipLaunchKernelGGL(grid_blocks, dim3((unsigned)((npts + 63) / 64)), dim3(64), 0, st, pts, npts, bsph);
}

void launch_grid_rho(int la, int lb, const CPair *cp, int ncp, const PrimPair *pp, const double4 *psph,
                     const double *xyz, const double *D, int ld, const double *pts, int64_t npts,
                     const double4 *bsph, double *rho, double *grad, hipStream_t st)
{
    if (ncp <= 0 || npts <= 0) return;
    const dim3 grid((unsigned)((npts + 63) / 64));
#define MD_GR(A_, B_)                                                                                        \
    if (la == A_ && lb == B_) {                                                                              \
        if (grad)                                                                                            \
            hipLaunchKernelGGL((grid_rho<A_, B_, true>), grid, dim3(64), 0, st, cp, ncp, pp, psph, xyz, D, ld, \
                               pts, npts, bsph, rho, grad);                                                  \
        else                                                                                                 \
            hipLaunchKernelGGL((grid_rho<A_, B_, false>), grid, dim3(64), 0, st, cp, ncp, pp, psph, xyz, D,   \
                               ld, pts, npts, bsph, rho, grad);                                              \
        return;                                                                                              \
    }
    MD_GR(0, 0) MD_GR(1, 0) MD_GR(1, 1) MD_GR(2, 0) MD_GR(2, 1) MD_GR(2, 2) MD_GR(3, 0) MD_GR(3, 1)
    MD_GR(3, 2) MD_GR(3, 3)
#undef MD_GR
}

void launch_grid_vmat(int la, int lb, const CPair *cp, int ncp, const PrimPair *pp, const double4 *psph,
                      const double *xyz, const double *pts, int64_t npts, const double4 *bsph, const double *v0,
                      const double *v1, double *Vacc, int ld, hipStream_t st)
{
    if (ncp <= 0 || npts <= 0) return;
    const int nblk = (int)((npts + 63) / 64);
#define MD_GV(A_, B_)                                                                                        \
    if (la == A_ && lb == B_) {                                                                              \
        if (v1)                                                                                              \
            hipLaunchKernelGGL((grid_vmat<A_, B_, true>), dim3((unsigned)ncp), dim3(64), 0, st, cp, ncp, pp,  \
                               psph, xyz, pts, npts, nblk, bsph, v0, v1, Vacc, ld);                          \
        else                                                                                                 \
            hipLaunchKernelGGL((grid_vmat<A_, B_, false>), dim3((unsigned)ncp), dim3(64), 0, st, cp, ncp, pp, \
                               psph, xyz, pts, npts, nblk, bsph, v0, v1, Vacc, ld);                          \
        return;                                                                                              \
    }
    MD_GV(0, 0) MD_GV(1, 0) MD_GV(1, 1) MD_GV(2, 0) MD_GV(2, 1) MD_GV(2, 2) MD_GV(3, 0) MD_GV(3, 1)
    MD_GV(3, 2) MD_GV(3, 3)
#undef MD_GV
}

}  // namespace md
