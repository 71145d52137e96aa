// eprod.hip -- Hermite expansion products of every primitive pair, computed
// once per geometry (they depend only on the pair, eq. E_recursion):
//   E^{ab}_t = E^{ax bx}_{tx} E^{ay by}_{ty} E^{az bz}_{tz},  t in box(ab),
// stored per pair as [ab][tx][ty][tz] (ab-major, tz fastest).  Exchange
// kernels read the bra products through wave-uniform loads.
#include "kern_args.hpp"
#include "launch.hpp"
#include "md_device.hpp"

namespace md {

template <int LA, int LB>
struct EprodLayout {
    static constexpr int NA = ncart(LA), NB = ncart(LB), NAB = NA * NB;
    int off[NAB + 1];
    constexpr EprodLayout() : off()
    {
        int o = 0;
        for (int ab = 0; ab < NAB; ++ab) {
            off[ab] = o;
            o += box_nnz(LA, ab / NB, LB, ab % NB);
        }
        off[NAB] = o;
    }
};

template <int LA, int LB, typename T>
__global__ __launch_bounds__(128) void eprod_build(const PrimPair *__restrict__ pp, int pbase, int n,
                                                   T *__restrict__ out)
{
    constexpr EprodLayout<LA, LB> lay{};
    constexpr int S = lay.off[lay.NAB];
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const PrimPair p = pp[pbase + g];
    Etab<LA, LB> Ex, Ey, Ez;
    etab_build<LA, LB>(p.PA[0], p.PB[0], p.o2p, Ex);
    etab_build<LA, LB>(p.PA[1], p.PB[1], p.o2p, Ey);
    etab_build<LA, LB>(p.PA[2], p.PB[2], p.o2p, Ez);
    T *o = out + (int64_t)g * S;
    // single precision: K_ab E_t (2p)^{|t|/2} (scaled form, md_device.hpp)
    double cw[LA + LB + 1];
    cw[0] = sizeof(T) == 4 ? p.K : 1.0;
    for (int k = 1; k <= LA + LB; ++k) cw[k] = cw[k - 1] * (sizeof(T) == 4 ? sqrt(2.0 * p.p) : 1.0);
    static_for<0, lay.NAB>([&](auto abc) {
        constexpr int ab = decltype(abc)::value;
        constexpr int a = ab / lay.NB, b = ab % lay.NB;
        constexpr int ax = cart_x(LA, a), ay = cart_y(LA, a), az = cart_z(LA, a);
        constexpr int bx = cart_x(LB, b), by = cart_y(LB, b), bz = cart_z(LB, b);
        constexpr int ny = ay + by + 1, nz = az + bz + 1;
        static_for<0, ax + bx + 1>([&](auto txc) {
            constexpr int tx = decltype(txc)::value;
            static_for<0, ny>([&](auto tyc) {
                constexpr int ty = decltype(tyc)::value;
                static_for<0, nz>([&](auto tzc) {
                    constexpr int tz = decltype(tzc)::value;
                    o[lay.off[ab] + (tx * ny + ty) * nz + tz] = (T)(Ex.e[ax][bx][tx] * Ey.e[ay][by][ty] * Ez.e[az][bz][tz] * cw[tx + ty + tz]);
                });
            });
        });
    });
}

int eprod_size(int la, int lb)
{
    int s = 0;
    for (int a = 0; a < ncart(la); ++a)
        for (int b = 0; b < ncart(lb); ++b) s += box_nnz(la, a, lb, b);
    return s;
}

// The products are formed in double precision; the single-precision table
// used by the mixed mode holds the scaled products K_ab E_t (2p)^{|t|/2}.
template <typename T>
void launch_eprod_t(int la, int lb, const PrimPair *pp, int pbase, int n, T *out, hipStream_t st)
{
    if (n <= 0) return;
    const unsigned blocks = (unsigned)((n + 127) / 128);
#define MD_EP(A_, B_)                                                                         \
    if (la == A_ && lb == B_) {                                                              \
        hipLaunchKernelGGL((eprod_build<A_, B_, T>), dim3(blocks), dim3(128), 0, st, pp, pbase, n, out); \
        return;                                                                              \
    }
    MD_EP(0, 0) MD_EP(1, 0) MD_EP(1, 1) MD_EP(2, 0) MD_EP(2, 1) MD_EP(2, 2) MD_EP(3, 0) MD_EP(3, 1)
    MD_EP(3, 2) MD_EP(3, 3)
#undef MD_EP
}

void launch_eprod(int la, int lb, const PrimPair *pp, int pbase, int n, double *out, hipStream_t st)
{
    launch_eprod_t<double>(la, lb, pp, pbase, n, out, st);
}

void launch_eprod(int la, int lb, const PrimPair *pp, int pbase, int n, float *out, hipStream_t st)
{
    launch_eprod_t<float>(la, lb, pp, pbase, n, out, st);
}

}  // namespace md
