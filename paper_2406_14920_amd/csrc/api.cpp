// api.cpp -- host implementation of the C ABI declared in include/mdjk.h.
//
// Setup (eri_setup): shells are normalised (contracted basis of
// eqs. contracted_basis / primtive_basis), contracted and primitive shell
// pairs are formed (eq. pair_definition) with the larger angular momentum
// first, Schwarz factors are computed on the GPU (eq. cauchy_schwarz_bound),
// pairs that cannot pass the quartet rule are dropped, the rest are sorted by
// bound inside the ten angular pair classes (primitive pairs by their own bound
// inside each contracted pair), and the exchange work lists are built: for a
// bra pair i of class X and ket class Y <= X the kets j with Q_i Q_j >= tau
// form a prefix of the sorted list.
//
// build_jk: P_sph -> P_cart, Hermite density, J-engine, Hermite -> Cartesian,
// exchange classes, and Cartesian accumulators -> (symmetrised) J and K.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/mdjk.h"
#include "class_lists.hpp"
#include "grid.hpp"
#include "launch.hpp"
#include "md_common.hpp"
#include "queue.hpp"

using namespace md;

namespace {

thread_local std::string g_err;

int set_err(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

struct HipError {
    int code;
};

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) {                                                               \
            set_err(e_ == hipErrorOutOfMemory ? ERI_ENOMEM : ERI_EHIP, "%s failed: %s (%s:%d)", #expr, \
                    hipGetErrorString(e_), __FILE__, __LINE__);                               \
            throw HipError{e_ == hipErrorOutOfMemory ? ERI_ENOMEM : ERI_EHIP};                \
        }                                                                                     \
    } while (0)

constexpr int kPairClasses = 10;
constexpr int kPairL[kPairClasses][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1},
                                         {2, 2}, {3, 0}, {3, 1}, {3, 2}, {3, 3}};
int pair_class(int la, int lb) { return la * (la + 1) / 2 + lb; }

bool uses_k_pair(int la, int lb, int lc, int ld)
{
#define MD_IS(A_, B_, C_, D_) if (la == A_ && lb == B_ && lc == C_ && ld == D_) return true;
    MD_K_PAIR_PART0(MD_IS) MD_K_PAIR_PART1(MD_IS) MD_K_PAIR_PART2(MD_IS) MD_K_PAIR_PART3(MD_IS)
    MD_K_PAIR_PART4(MD_IS) MD_K_PAIR_PART5(MD_IS) MD_K_PAIR_PART6(MD_IS) MD_K_PAIR_PART7(MD_IS)
#undef MD_IS
    return false;
}

// ---------------------------------------------------------------------------
// Algorithmic FLOP model (frozen before tuning):
//   Boys 3L+14, R 3(C(L+4,4)-(L+1)) + (L+1) per primitive quartet,
//   K contraction sum_cd 2 nH(la+lb) nnz(cd) + sum_{ab,cd} 2 nnz(ab) per
//   primitive quartet and 8 nA nB nC nD digestion per shell quartet,
//   J-engine 2 nH(LX) nH(LY) per (bra, ket) primitive pair.
// ---------------------------------------------------------------------------
double binom4(int n) { return n < 4 ? 0.0 : (double)n * (n - 1) * (n - 2) * (n - 3) / 24.0; }
double fl_boys(int L) { return 3.0 * L + 14.0; }
double fl_r(int L) { return 3.0 * (binom4(L + 4) - (L + 1)) + (L + 1); }
double sum_nnz(int la, int lb)
{
    double s = 0.0;
    for (int a = 0; a < ncart(la); ++a)
        for (int b = 0; b < ncart(lb); ++b) s += box_nnz(la, a, lb, b);
    return s;
}
double fl_k_prim(int la, int lb, int lc, int ld)
{
    const int L = la + lb + lc + ld;
    return fl_boys(L) + fl_r(L) + 2.0 * nherm(la + lb) * sum_nnz(lc, ld) +
           2.0 * ncart(lc) * ncart(ld) * sum_nnz(la, lb);
}
double fl_k_digest(int la, int lb, int lc, int ld) { return 8.0 * ncart(la) * ncart(lb) * ncart(lc) * ncart(ld); }
double fl_j_prim(int lx, int ly) { return fl_boys(lx + ly) + fl_r(lx + ly) + 2.0 * nherm(lx) * nherm(ly); }
// one (primitive pair, point charge) term of the Hermite potential of order L:
// distance and Boys argument, Boys, the scaled R^m_000, R, the accumulation
double fl_v(int L) { return 8.0 + fl_boys(L) + fl_r(L) + 2.0 * (L + 1) + nherm(L); }
// one (primitive pair, charge) term of the charge derivative at pair order L
double fl_vg(int L) { return 8.0 + fl_boys(L + 1) + fl_r(L + 1) + 2.0 * (L + 2) + 7.0 * nherm(L); }

bool jeng_is_reg(int lx, int ly)
{
    return lx + ly >= 6 && nherm(lx) + 4 * (lx + ly + 1) + (nherm(ly) <= 20 ? nherm(ly) : 0) <= 116;
}

// Default ket chunk of a J-engine launch: the largest power of two in
// [8, 256] that still gives the launch at least 16384 workgroups (one per
// bra primitive pair, or per 64 of them, times the ket chunks), so that the
// classes with few bra primitive pairs fill the 256 CUs instead of running
// long ket loops on a few hundred waves.
int jeng_default_chunk(int lx, int ly, int npp, int ncp)
{
    const bool per_pair = lx + ly > 5 && !jeng_is_reg(lx, ly);
    const int64_t nx = per_pair ? npp : (npp + 63) / 64;
    int kc = 256;
    while (kc > 8 && nx * ((ncp + kc - 1) / kc) < 16384) kc /= 2;
    return kc;
}

// ---------------------------------------------------------------------------
// Boys table: F_m(i h) for m < kBoysNM, then e^{-i h}.  For each grid point the top order
// (m = 60) is summed from its Kummer series e^{-T} sum_k (2T)^k/(2m+1)...(2m+2k+1)
// in long double, then every lower order follows from the downward recursion
// F_m = (2T F_{m+1} + e^{-T})/(2m+1), which is stable.
// ---------------------------------------------------------------------------
const std::vector<double> &boys_table()
{
    static std::vector<double> tab;
    static std::once_flag once;
    std::call_once(once, [] {
        const int top = 60;
        tab.assign((size_t)kBoysNG * kBoysNC, 0.0);
        for (int i = 0; i < kBoysNG; ++i) {
            long double T = (long double)i * (long double)kBoysH;
            long double eT = expl(-T);
            long double term = 1.0L / (2 * top + 1), sum = term;
            for (int k = 1; k < 4000; ++k) {
                term *= 2.0L * T / (long double)(2 * top + 2 * k + 1);
                sum += term;
                if (term < 1e-22L * sum) break;
            }
            long double F = eT * sum;
            for (int m = top - 1; m >= 0; --m) {
                F = (2.0L * T * F + eT) / (long double)(2 * m + 1);
                if (m < kBoysNM) tab[(size_t)i * kBoysNC + m] = (double)F;
            }
            tab[(size_t)i * kBoysNC + kBoysNM] = (double)eT;
        }
    });
    return tab;
}

double dfact(int n)
{
    double r = 1.0;
    for (; n > 1; n -= 2) r *= n;
    return r;
}

// Device bytes held by the library's buffers in this process, and the cap
// that the environment variable ERI_MAX_DEVICE_BYTES may set (read at every
// allocation; unset or 0: none) so that tests can drive the out-of-memory
// paths without exhausting the device.
std::atomic<unsigned long long> g_dev_bytes{0};

unsigned long long dev_cap()
{
    const char *s = std::getenv("ERI_MAX_DEVICE_BYTES");
    return s ? std::strtoull(s, nullptr, 10) : 0ull;
}

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    void alloc(size_t count)
    {
        release();
        if (count) {
            const unsigned long long bytes = (unsigned long long)count * sizeof(T), cap = dev_cap();
            if (cap && g_dev_bytes.load() + bytes > cap) {
                set_err(ERI_ENOMEM, "device allocation of %llu bytes would pass ERI_MAX_DEVICE_BYTES=%llu (%llu held)",
                        bytes, cap, (unsigned long long)g_dev_bytes.load());
                throw HipError{ERI_ENOMEM};
            }
            HIPCHK(hipMalloc((void **)&p, count * sizeof(T)));
            g_dev_bytes += bytes;
        }
        n = count;
    }
    void upload(const std::vector<T> &h)
    {
        alloc(h.size());
        if (!h.empty()) HIPCHK(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    }
    void release()
    {
        if (p) {
            (void)hipFree(p);
            g_dev_bytes -= (unsigned long long)n * sizeof(T);
        }
        p = nullptr;
        n = 0;
    }
    ~DevBuf() { release(); }
};

}  // namespace

struct eri_ctx {
    uint32_t magic = 0x4d444a4b;
    uint64_t gen = 0;  // bumped by every change that invalidates captured graphs
    eri_opts opts{};
    hipStream_t st = nullptr;
    int device = 0;

    // basis (host)
    int nshell = 0, natom = 0, nbf = 0, nbf_cart = 0;
    std::vector<int32_t> sh_atom, sh_l, sh_np, sh_poff, sh_coff, sh_soff;
    std::vector<double> pexp, pcoef, xyz;

    // pairs (host, final order)
    int ncp[kPairClasses] = {}, cp_base[kPairClasses] = {};
    int npp[kPairClasses] = {}, pp_base[kPairClasses] = {};
    std::vector<CPair> cp;
    std::vector<double> Q;
    std::vector<PrimPair> pp;
    // exchange work lists for (X >= Y)
    struct KWork {
        int X, Y;
        int64_t off;    // into prefix buffer
        int64_t nwork;
        int64_t choff;  // into chunk buffer (bra-shared kernel), -1 if unused
        int nchunks;
        int64_t roff;   // into row buffer
        int nrows;
    };
    // exchange views: per class the pairs grouped by contraction length
    // (largest first) and by one shell -- view 0 the first shell c, view 1
    // the second shell d -- Q descending inside a group (same class bases as
    // cp); vorig maps a view index to the Q-order index inside the class,
    // kgroups lists each class's groups (first, count) in view order
    std::vector<CPair> kcp[2];
    std::vector<double> kQ[2];
    std::vector<int> vorig[2];
    std::vector<std::vector<std::array<int, 2>>> kgroups[2];
    std::vector<KWork> kwork;
    std::vector<int> kinv;  // per exchange launch: the view its kets come from
    double tau_dens = 0.0;  // density-weighted screen of build_jk (0: off)
    size_t dt_off[kPairClasses] = {}, jh_off[kPairClasses] = {};

    // device
    DevBuf<CPair> d_cp;
    DevBuf<double> d_Q;
    DevBuf<PrimPair> d_pp;
    DevBuf<int32_t> d_owner;
    DevBuf<int64_t> d_prefix;
    DevBuf<int2> d_rows;
    DevBuf<CPair> d_kcp[2];
    DevBuf<double> d_kQ[2];
    DevBuf<int4> d_chunks;
    DevBuf<double> d_eprod;
    size_t eprod_off[kPairClasses] = {};
    DevBuf<double> d_boys;
    DevBuf<double> d_Pc, d_Jacc, d_Kacc, d_Dt, d_Jh;
    // the per-build work buffers the kernels are handed: the context's own
    // (above), or regions of the static scratch array during build_jk_static
    struct Work {
        double *Pc = nullptr, *Jacc = nullptr, *Kacc = nullptr, *Dt = nullptr, *Jh = nullptr;
    } wk;
    DevBuf<int32_t> d_soc, d_sos, d_l, d_coff, d_soff;

    // mixed precision: single-precision Hermite products and Hermite density
    // (built on first use after each geometry), shell-pair density bounds and
    // Q max|D| per contracted pair (per build)
    bool mixed_ready = false;
    DevBuf<float> d_eprodf, d_Dtf;
    DevBuf<double> d_Pm, d_QD;
    bool built_mixed = false;  // last build_jk ran in the mixed mode
    // single-precision share of the last mixed build: per exchange launch and
    // per J-engine (X, Y): {primitive quartets, work items}; computed on demand
    mutable bool mix_counts_ok = false;
    mutable std::vector<std::array<int64_t, 2>> kmix;
    mutable int64_t jmix[kPairClasses][kPairClasses][2] = {};

    // gradient: Hermite J of order LX+1, per-pair Coulomb terms, exchange
    // workgroup partials (allocated on the first jk_grad after each geometry)
    bool grad_ready = false, jh1_ready = false;
    size_t jh1_off[kPairClasses] = {};
    DevBuf<double> d_vpart;  // charge-gradient partials of eri_potential_grad
    // grid integrals: atom positions, bounding sphere of every contracted pair
    // (J order), bounding spheres of the current call's point blocks
    bool grid_ready = false;
    DevBuf<double> d_xyz;
    DevBuf<double4> d_psph, d_bsph;
    DevBuf<double> d_gpart;  // per-stream density partials of eri_grid_density
    DevBuf<double> d_Jh1, d_pg, d_kpart, d_Jtmp, d_Ktmp, d_jhpart;
    DevBuf<double> d_gred;  // chunk sums of the fixed-order gradient reduction
    int gchunk[kPairClasses][kPairClasses] = {};  // J-engine ket chunk of the gradient launches
    std::vector<int> kg_blocks;   // per exchange launch
    std::vector<int64_t> kg_off;  // first partial of each launch
    int64_t kg_total = 0;

    // primitive-quartet counts per exchange launch and per J-engine (X, Y)
    std::vector<int64_t> kprim;
    int64_t jprim[kPairClasses][kPairClasses] = {};

    // profiling: work = {-1 none, 0 exchange launch, 1 J-engine}, idx = kwork
    // index or X*10+Y, part = 0 whole launch, 1 double / 2 single share
    struct Rec {
        std::string name;
        hipEvent_t a, b;
        int work, idx, part;
    };
    struct Acc {
        int launches = 0;
        double ms = 0, flops = 0;
        int64_t pq = 0;
    };
    // launch-shape parameters (set by eri_autotune): J-engine ket chunk per
    // (bra class, ket class) and workgroup cap per exchange launch
    int kchunk[kPairClasses][kPairClasses];
    std::vector<int> kcap;
    // ERI_MIXED: whether a launch takes the single-precision share at all
    // (J-engine per (X, Y), exchange per work list); ERI_MIXED_ALL splits all
    bool jsplit[kPairClasses][kPairClasses];
    std::vector<char> ksplit;

    bool profile = false;
    std::vector<Rec> pending;
    // streams the J work and the bra-shared / small exchange launches fork
    // onto, joined back into the context stream by events
    bool recording = false;  // inside a batch graph recording: no internal fork
    hipStream_t aux[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_kzero = nullptr, ev_join[3] = {nullptr, nullptr, nullptr};
    std::map<std::string, Acc> prof;

    // stats
    int64_t n_quartets = 0;
    double eris_sph = 0, eris_cart = 0;
    double model_flops_k = 0, model_flops_j = 0;
    double last_ms = 0;
};

namespace {

int validate(const eri_shell *shells, int32_t nshell, const eri_atom *atoms, int32_t natom,
             const eri_opts *o)
{
    if (!shells || !atoms || nshell <= 0 || natom <= 0)
        return set_err(ERI_EINVAL, "null shells/atoms or non-positive counts (nshell=%d, natom=%d)", nshell, natom);
    for (int i = 0; i < natom; ++i)
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(atoms[i].xyz[k])) return set_err(ERI_EINVAL, "atom %d coordinate not finite", i);
    for (int s = 0; s < nshell; ++s) {
        const eri_shell &sh = shells[s];
        if (sh.l < 0 || sh.l > 3) return set_err(ERI_EINVAL, "shell %d: l=%d outside 0..3", s, sh.l);
        if (sh.nprim < 1) return set_err(ERI_EINVAL, "shell %d: nprim=%d < 1", s, sh.nprim);
        if (sh.atom < 0 || sh.atom >= natom)
            return set_err(ERI_EINVAL, "shell %d: atom index %d out of range", s, sh.atom);
        if (!sh.exps || !sh.coefs) return set_err(ERI_EINVAL, "shell %d: null exps/coefs", s);
        for (int k = 0; k < sh.nprim; ++k) {
            if (!(sh.exps[k] > 0.0) || !std::isfinite(sh.exps[k]))
                return set_err(ERI_EINVAL, "shell %d: exponent %d = %g not positive and finite", s, k, sh.exps[k]);
            if (!std::isfinite(sh.coefs[k])) return set_err(ERI_EINVAL, "shell %d: coefficient %d not finite", s, k);
        }
    }
    if (o) {
        if (!(o->schwarz_thresh >= 0.0) || !(o->prim_thresh >= 0.0) || !(o->mixed_thresh >= 0.0))
            return set_err(ERI_EINVAL, "negative or NaN threshold");
        if (o->precision != ERI_FP64 && o->precision != ERI_MIXED && o->precision != ERI_MIXED_ALL)
            return set_err(ERI_EINVAL, "unknown precision %d", o->precision);
        if (!(o->omega >= 0.0) || !std::isfinite(o->omega))
            return set_err(ERI_EINVAL, "omega %g not non-negative and finite", o->omega);
    }
    return ERI_OK;
}

// Contraction coefficients times primitive normalisation, rescaled so that
// the x^l component of the contracted shell has unit norm.  The self-overlap
// of two primitives on one centre is prod over x,y,z of the 1D Gaussian
// moments: int x^{2l} e^{-p x^2} dx * (int e^{-p x^2} dx)^2.
void normalise_shell(int l, int np, const double *e, const double *c, double *out)
{
    for (int k = 0; k < np; ++k) {
        const double a = e[k];
        const double N = std::pow(2.0 * a / kPi, 0.75) * std::pow(4.0 * a, 0.5 * l) / std::sqrt(dfact(2 * l - 1));
        out[k] = c[k] * N;
    }
    double S = 0.0;
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
            const double p = e[i] + e[j];
            const double g0 = std::sqrt(kPi / p);
            const double g2l = dfact(2 * l - 1) / std::pow(2.0 * p, l) * g0;  // int x^{2l} e^{-p x^2}
            S += out[i] * out[j] * g2l * g0 * g0;
        }
    const double f = 1.0 / std::sqrt(S);
    for (int k = 0; k < np; ++k) out[k] *= f;
}

void make_prim_pair(PrimPair &r, double a, double b, double ca, double cb, const double *A, const double *B)
{
    r.a = a;
    r.b = b;
    r.p = a + b;
    r.o2p = 0.5 / r.p;
    double ab2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        r.P[k] = (a * A[k] + b * B[k]) / r.p;
        r.PA[k] = r.P[k] - A[k];
        r.PB[k] = r.P[k] - B[k];
        ab2 += (A[k] - B[k]) * (A[k] - B[k]);
    }
    r.K = ca * cb * std::exp(-a * b / r.p * ab2);
    r.q = 0.0;
    r.pad = 0.0;
}

// The exchange kernels see each class through a view grouped by
// contraction length and by one shell of the pair, Q-sorted inside a group.
// A row of a work list pairs one bra with the kets of one group; the kets it
// visits (Q_i Q_j >= tau and, in a class with itself, j not after i in the Q
// order) form a prefix of the group.  Rows run bra by bra, so neighbouring
// work items share the bra and, inside a row, the grouping shell: with view 0
// (grouped by the first shell c of a ket (cd|)) their exchange contributions
// K_ac and K_bc go to the same elements, with view 1 (grouped by d) K_ad and
// K_bd do, and the kernels sum those across the lanes before one atomic
// addition per element (view 1 is what the paper calls the inverted
// ordering).  The length (the number of primitive pairs rounded up to a power
// of two, largest first) keeps the primitive loops of neighbouring lanes
// equally long.
void build_views(eri_ctx *c)
{
    auto np_group = [](int np) {
        int g = 0;
        while ((1 << g) < np) ++g;
        return g;
    };
    for (int v = 0; v < 2; ++v) {
        auto sh = [v](const CPair &x) { return v == 0 ? x.sh1 : x.sh2; };
        auto key_less = [&](const CPair &x, const CPair &y) {
            const int gx = np_group(x.np), gy = np_group(y.np);
            return gx != gy ? gx > gy : sh(x) < sh(y);
        };
        auto key_same = [&](const CPair &x, const CPair &y) {
            return np_group(x.np) == np_group(y.np) && sh(x) == sh(y);
        };
        c->kcp[v].assign(c->cp.size(), CPair{});
        c->kQ[v].assign(c->cp.size(), 0.0);
        c->vorig[v].assign(c->cp.size(), 0);
        c->kgroups[v].assign(kPairClasses, {});
        for (int X = 0; X < kPairClasses; ++X) {
            const int b = c->cp_base[X], nX = c->ncp[X];
            std::vector<int> idx(nX);
            for (int k = 0; k < nX; ++k) idx[k] = k;
            std::stable_sort(idx.begin(), idx.end(),
                             [&](int x, int y) { return key_less(c->cp[b + x], c->cp[b + y]); });
            for (int r = 0; r < nX; ++r) {
                c->kcp[v][b + r] = c->cp[b + idx[r]];
                c->kQ[v][b + r] = c->Q[b + idx[r]];
                c->vorig[v][b + r] = idx[r];
                if (r == 0 || !key_same(c->cp[b + idx[r]], c->cp[b + idx[r - 1]])) c->kgroups[v][X].push_back({r, 0});
                c->kgroups[v][X].back()[1]++;
            }
        }
        c->d_kcp[v].upload(c->kcp[v]);
        c->d_kQ[v].upload(c->kQ[v]);
    }
}

bool is_k_small(int la, int lb, int lc, int ld)
{
#define MD_IS(A_, B_, C_, D_) if (la == A_ && lb == B_ && lc == C_ && ld == D_) return true;
    MD_K_SMALL_LIST(MD_IS)
#undef MD_IS
    return false;
}

// Whether an exchange launch may take its kets from view 1 (the kernels with
// a lane per work item; the LDS kernels keep per-row tiles of K_ac and K_bc).
bool kinv_ok(int X, int Y)
{
    const int la = kPairL[X][0], lb = kPairL[X][1], lc = kPairL[Y][0], ld = kPairL[Y][1];
    return uses_k_pair(la, lb, lc, ld) || is_k_small(la, lb, lc, ld);
}

// Exchange work lists of every launch (X >= Y) from the view each one uses.
void build_kwork(eri_ctx *c)
{
    const double tau = c->opts.schwarz_thresh;
    std::vector<int64_t> prefix;
    std::vector<int2> rows;
    std::vector<int4> chunks;
    c->kwork.clear();
    c->n_quartets = 0;
    c->eris_sph = c->eris_cart = 0.0;
    for (int X = 0; X < kPairClasses; ++X)
        for (int Y = 0; Y <= X; ++Y) {
            const int v = c->kinv[c->kwork.size()] && kinv_ok(X, Y) ? 1 : 0;
            c->kinv[c->kwork.size()] = v;
            const std::vector<double> &kQ = c->kQ[v];
            const std::vector<int> &vorig = c->vorig[v];
            eri_ctx::KWork w{X, Y, (int64_t)prefix.size(), 0, -1, 0, (int64_t)rows.size(), 0};
            const int bX = c->cp_base[X], bY = c->cp_base[Y];
            const bool kp = uses_k_pair(kPairL[X][0], kPairL[X][1], kPairL[Y][0], kPairL[Y][1]);
            if (kp) w.choff = (int64_t)chunks.size();
            int64_t acc = 0;
            prefix.push_back(0);
            for (int i = 0; i < c->ncp[X]; ++i) {
                const double Qi = kQ[bX + i];
                const int oi = vorig[bX + i];
                const int r_first = (int)((int64_t)rows.size() - w.roff);
                const int64_t w_first = acc;
                for (const auto &gy : c->kgroups[v][Y]) {
                    const int j0 = gy[0], j1 = gy[0] + gy[1];
                    int lo = j0, hi = j1;  // Q descending inside the group
                    while (lo < hi) {
                        const int mid = (lo + hi) / 2;
                        if (Qi * kQ[bY + mid] >= tau) lo = mid + 1; else hi = mid;
                    }
                    int cnt = lo - j0;
                    if (X == Y) {  // Q-order index ascending inside the group
                        int l2 = j0, h2 = j0 + cnt;
                        while (l2 < h2) {
                            const int mid = (l2 + h2) / 2;
                            if (vorig[bY + mid] <= oi) l2 = mid + 1; else h2 = mid;
                        }
                        cnt = l2 - j0;
                    }
                    if (cnt <= 0) continue;
                    rows.push_back(make_int2(i, j0));
                    acc += cnt;
                    prefix.push_back(acc);
                }
                // bra-shared chunks: 64 consecutive work items of this bra
                // (first row, offset in it, items, rows spanned)
                if (kp) {
                    const int r_end = (int)((int64_t)rows.size() - w.roff);
                    int r = r_first;
                    for (int64_t s0 = w_first; s0 < acc; s0 += 64) {
                        const int64_t s1 = std::min<int64_t>(s0 + 64, acc);
                        while (prefix[w.off + r + 1] <= s0) ++r;
                        int r1 = r;
                        while (r1 + 1 < r_end && prefix[w.off + r1 + 1] < s1) ++r1;
                        chunks.push_back(make_int4(r, (int)(s0 - prefix[w.off + r]), (int)(s1 - s0), r1 - r + 1));
                    }
                }
            }
            w.nwork = acc;
            w.nrows = (int)((int64_t)rows.size() - w.roff);
            if (kp) w.nchunks = (int)((int64_t)chunks.size() - w.choff);
            c->kwork.push_back(w);
            c->n_quartets += acc;
            const int la = kPairL[X][0], lb = kPairL[X][1], lc = kPairL[Y][0], ld = kPairL[Y][1];
            c->eris_sph += (double)acc * nsph(la) * nsph(lb) * nsph(lc) * nsph(ld);
            c->eris_cart += (double)acc * ncart(la) * ncart(lb) * ncart(lc) * ncart(ld);
        }
    c->d_prefix.upload(prefix);
    c->d_rows.upload(rows);
    c->d_chunks.upload(chunks);
    c->mix_counts_ok = false;
    ++c->gen;
}

// Build pairs, run the Schwarz kernels, sort, build the work lists.
void build_pairs(eri_ctx *c)
{
    const double tau = c->opts.schwarz_thresh;
    // 1. raw pairs grouped by class
    std::vector<CPair> rcp[kPairClasses];
    std::vector<std::vector<PrimPair>> rpp[kPairClasses];
    for (int s1 = 0; s1 < c->nshell; ++s1)
        for (int s2 = 0; s2 <= s1; ++s2) {
            int a = s1, b = s2;
            if (c->sh_l[b] > c->sh_l[a]) std::swap(a, b);
            const int X = pair_class(c->sh_l[a], c->sh_l[b]);
            CPair cpr{};
            cpr.sh1 = a;
            cpr.sh2 = b;
            cpr.c1 = c->sh_coff[a];
            cpr.c2 = c->sh_coff[b];
            cpr.at1 = c->sh_atom[a];
            cpr.at2 = c->sh_atom[b];
            const double *A = &c->xyz[3 * c->sh_atom[a]];
            const double *B = &c->xyz[3 * c->sh_atom[b]];
            std::vector<PrimPair> prims;
            for (int i = 0; i < c->sh_np[a]; ++i)
                for (int j = 0; j < c->sh_np[b]; ++j) {
                    PrimPair r;
                    make_prim_pair(r, c->pexp[c->sh_poff[a] + i], c->pexp[c->sh_poff[b] + j],
                                   c->pcoef[c->sh_poff[a] + i], c->pcoef[c->sh_poff[b] + j], A, B);
                    prims.push_back(r);
                }
            rcp[X].push_back(cpr);
            rpp[X].push_back(std::move(prims));
        }
    // 2. upload unsorted and compute Schwarz factors
    std::vector<CPair> ucp;
    std::vector<PrimPair> upp;
    int ubase[kPairClasses], un[kPairClasses];
    for (int X = 0; X < kPairClasses; ++X) {
        ubase[X] = (int)ucp.size();
        un[X] = (int)rcp[X].size();
        for (size_t k = 0; k < rcp[X].size(); ++k) {
            CPair cpr = rcp[X][k];
            cpr.poff = (int)upp.size();
            cpr.np = (int)rpp[X][k].size();
            ucp.push_back(cpr);
            upp.insert(upp.end(), rpp[X][k].begin(), rpp[X][k].end());
        }
    }
    DevBuf<CPair> ucp_d;
    DevBuf<PrimPair> upp_d;
    DevBuf<double> uQ_d;
    ucp_d.upload(ucp);
    upp_d.upload(upp);
    uQ_d.alloc(ucp.size());
    for (int X = 0; X < kPairClasses; ++X)
        launch_schwarz(kPairL[X][0], kPairL[X][1], ucp_d.p + ubase[X], un[X], upp_d.p, uQ_d.p + ubase[X],
                       c->d_boys.p, c->st);
    HIPCHK(hipGetLastError());
    std::vector<double> uQ(ucp.size());
    HIPCHK(hipStreamSynchronize(c->st));
    HIPCHK(hipMemcpy(uQ.data(), uQ_d.p, uQ.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(upp.data(), upp_d.p, upp.size() * sizeof(PrimPair), hipMemcpyDeviceToHost));
    double Qmax = 0.0;
    for (double v : uQ) Qmax = std::max(Qmax, v);

    // 3. drop pairs that can never pass, sort by Q, sort primitives by q
    c->cp.clear();
    c->Q.clear();
    c->pp.clear();
    std::vector<int32_t> owner;
    for (int X = 0; X < kPairClasses; ++X) {
        std::vector<int> idx;
        for (int k = 0; k < un[X]; ++k) {
            const double q = uQ[ubase[X] + k];
            if (q > 0.0 && q * Qmax >= tau) idx.push_back(k);
        }
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return uQ[ubase[X] + x] > uQ[ubase[X] + y]; });
        c->cp_base[X] = (int)c->cp.size();
        c->ncp[X] = (int)idx.size();
        c->pp_base[X] = (int)c->pp.size();
        for (size_t r = 0; r < idx.size(); ++r) {
            CPair cpr = ucp[ubase[X] + idx[r]];
            std::vector<PrimPair> prims(upp.begin() + cpr.poff, upp.begin() + cpr.poff + cpr.np);
            std::stable_sort(prims.begin(), prims.end(), [](const PrimPair &u, const PrimPair &v) { return u.q > v.q; });
            cpr.poff = (int)c->pp.size();
            for (auto &pr : prims) {
                c->pp.push_back(pr);
                owner.push_back((int32_t)r);
            }
            c->cp.push_back(cpr);
            c->Q.push_back(uQ[ubase[X] + idx[r]]);
        }
        c->npp[X] = (int)c->pp.size() - c->pp_base[X];
    }
    c->d_cp.upload(c->cp);
    c->d_Q.upload(c->Q);
    c->d_pp.upload(c->pp);
    c->d_owner.upload(owner);
    c->d_QD.alloc(std::max<size_t>(c->cp.size(), 1));
    c->mixed_ready = false;
    c->built_mixed = false;
    c->mix_counts_ok = false;
    c->grad_ready = false;
    c->jh1_ready = false;
    c->grid_ready = false;

    // 4. exchange views and work lists (build_views, build_kwork)
    build_views(c);
    c->kinv.assign((size_t)kPairClasses * (kPairClasses + 1) / 2, 0);
    build_kwork(c);
    for (int X = 0; X < kPairClasses; ++X)
        for (int Y = 0; Y < kPairClasses; ++Y) {
            c->kchunk[X][Y] = jeng_default_chunk(kPairL[X][0] + kPairL[X][1], kPairL[Y][0] + kPairL[Y][1],
                                                 c->npp[X], c->ncp[Y]);
            c->jsplit[X][Y] = false;  // FP64 J-engine: Boys and conversions dominate its FP32 share
        }
    c->kcap.assign(c->kwork.size(), 0);
    c->ksplit.assign(c->kwork.size(), 0);
    for (size_t wi = 0; wi < c->kwork.size(); ++wi) {
        const auto &w = c->kwork[wi];
        c->ksplit[wi] = kPairL[w.X][0] + kPairL[w.X][1] + kPairL[w.Y][0] + kPairL[w.Y][1] >= 5;
    }

    // Hermite products of every primitive pair (bra/ket data of the bra-shared kernel)
    size_t ep = 0;
    for (int X = 0; X < kPairClasses; ++X) {
        c->eprod_off[X] = ep;
        ep += (size_t)c->npp[X] * eprod_size(kPairL[X][0], kPairL[X][1]);
    }
    c->d_eprod.alloc(std::max<size_t>(ep, 1));
    for (int X = 0; X < kPairClasses; ++X)
        launch_eprod(kPairL[X][0], kPairL[X][1], c->d_pp.p, c->pp_base[X], c->npp[X], c->d_eprod.p + c->eprod_off[X],
                     c->st);
    HIPCHK(hipGetLastError());

    // 5. Hermite density / Hermite J storage
    size_t dt = 0;
    for (int X = 0; X < kPairClasses; ++X) {
        c->dt_off[X] = dt;
        c->jh_off[X] = dt;
        dt += (size_t)c->npp[X] * nherm(kPairL[X][0] + kPairL[X][1]);
    }
    c->d_Dt.alloc(std::max<size_t>(dt, 1));
    c->d_Jh.alloc(std::max<size_t>(dt, 1));
    c->wk.Dt = c->d_Dt.p;
    c->wk.Jh = c->d_Jh.p;

    // 6. primitive quartets each launch evaluates (same loops as the kernels)
    const size_t ncount = c->kwork.size() + kPairClasses * kPairClasses;
    DevBuf<unsigned long long> cnt;
    cnt.alloc(ncount);
    HIPCHK(hipMemsetAsync(cnt.p, 0, ncount * sizeof(unsigned long long), c->st));
    for (size_t wi = 0; wi < c->kwork.size(); ++wi) {
        const auto &w = c->kwork[wi];
        KArgs a{};
        a.bra = c->d_kcp[c->kinv[wi]].p + c->cp_base[w.X];
        a.ket = c->d_kcp[c->kinv[wi]].p + c->cp_base[w.Y];
        a.rows = c->d_rows.p + w.roff;
        a.prefix = c->d_prefix.p + w.off;
        a.nwork = w.nwork;
        a.nrows = w.nrows;
        a.pp = c->d_pp.p;
        a.tau_prim = c->opts.prim_thresh;
        launch_k_count(a, cnt.p + wi, c->st);
    }
    for (int X = 0; X < kPairClasses; ++X)
        for (int Y = 0; Y < kPairClasses; ++Y) {
            JArgs a{};
            a.pp = c->d_pp.p;
            a.owner = c->d_owner.p + c->pp_base[X];
            a.Qbra = c->d_Q.p + c->cp_base[X];
            a.pbase = c->pp_base[X];
            a.nbp = c->npp[X];
            a.ket = c->d_cp.p + c->cp_base[Y];
            a.Qket = c->d_Q.p + c->cp_base[Y];
            a.nket = c->ncp[Y];
            a.tau = tau;
            a.tau_prim = c->opts.prim_thresh;
            launch_j_count(a, cnt.p + c->kwork.size() + X * kPairClasses + Y, c->st);
        }
    HIPCHK(hipGetLastError());
    std::vector<unsigned long long> hc(ncount);
    HIPCHK(hipStreamSynchronize(c->st));
    HIPCHK(hipMemcpy(hc.data(), cnt.p, ncount * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    c->kprim.assign(c->kwork.size(), 0);
    c->model_flops_k = 0.0;
    for (size_t wi = 0; wi < c->kwork.size(); ++wi) {
        const auto &w = c->kwork[wi];
        c->kprim[wi] = (int64_t)hc[wi];
        const int la = kPairL[w.X][0], lb = kPairL[w.X][1], lc = kPairL[w.Y][0], ld = kPairL[w.Y][1];
        c->model_flops_k += (double)hc[wi] * fl_k_prim(la, lb, lc, ld) + (double)w.nwork * fl_k_digest(la, lb, lc, ld);
    }
    c->model_flops_j = 0.0;
    for (int X = 0; X < kPairClasses; ++X)
        for (int Y = 0; Y < kPairClasses; ++Y) {
            c->jprim[X][Y] = (int64_t)hc[c->kwork.size() + X * kPairClasses + Y];
            c->model_flops_j += (double)c->jprim[X][Y] *
                                fl_j_prim(kPairL[X][0] + kPairL[X][1], kPairL[Y][0] + kPairL[Y][1]);
        }
}

void build_basis(eri_ctx *c, const eri_shell *shells, const eri_atom *atoms)
{
    c->sh_atom.resize(c->nshell);
    c->sh_l.resize(c->nshell);
    c->sh_np.resize(c->nshell);
    c->sh_poff.resize(c->nshell);
    c->sh_coff.resize(c->nshell);
    c->sh_soff.resize(c->nshell);
    c->pexp.clear();
    c->pcoef.clear();
    int co = 0, so = 0;
    for (int s = 0; s < c->nshell; ++s) {
        const eri_shell &sh = shells[s];
        c->sh_atom[s] = sh.atom;
        c->sh_l[s] = sh.l;
        c->sh_np[s] = sh.nprim;
        c->sh_poff[s] = (int)c->pexp.size();
        c->sh_coff[s] = co;
        c->sh_soff[s] = so;
        co += ncart(sh.l);
        so += c->opts.spherical ? nsph(sh.l) : ncart(sh.l);
        std::vector<double> nc(sh.nprim);
        normalise_shell(sh.l, sh.nprim, sh.exps, sh.coefs, nc.data());
        for (int k = 0; k < sh.nprim; ++k) {
            c->pexp.push_back(sh.exps[k]);
            c->pcoef.push_back(nc[k]);
        }
    }
    c->nbf_cart = co;
    c->nbf = so;
    c->xyz.resize(3 * c->natom);
    for (int i = 0; i < c->natom; ++i)
        for (int k = 0; k < 3; ++k) c->xyz[3 * i + k] = atoms[i].xyz[k];

    std::vector<int32_t> soc(c->nbf_cart), sos(c->nbf);
    for (int s = 0; s < c->nshell; ++s) {
        for (int k = 0; k < ncart(c->sh_l[s]); ++k) soc[c->sh_coff[s] + k] = s;
        const int ns = c->opts.spherical ? nsph(c->sh_l[s]) : ncart(c->sh_l[s]);
        for (int k = 0; k < ns; ++k) sos[c->sh_soff[s] + k] = s;
    }
    c->d_soc.upload(soc);
    c->d_sos.upload(sos);
    c->d_l.upload(c->sh_l);
    c->d_coff.upload(c->sh_coff);
    c->d_soff.upload(c->sh_soff);
    const size_t nc2 = (size_t)c->nbf_cart * c->nbf_cart;
    c->d_Pc.alloc(nc2);
    c->d_Jacc.alloc(nc2);
    c->d_Kacc.alloc(nc2);
    c->wk.Pc = c->d_Pc.p;
    c->wk.Jacc = c->d_Jacc.p;
    c->wk.Kacc = c->d_Kacc.p;
    c->d_Pm.alloc((size_t)c->nshell * c->nshell);
}

// Single-precision tables of the mixed mode (geometry dependent only).
void ensure_mixed(eri_ctx *c)
{
    if (c->mixed_ready) return;
    c->d_eprodf.alloc(std::max<size_t>(c->d_eprod.n, 1));
    for (int X = 0; X < kPairClasses; ++X)
        launch_eprod(kPairL[X][0], kPairL[X][1], c->d_pp.p, c->pp_base[X], c->npp[X],
                     c->d_eprodf.p + c->eprod_off[X], c->st);
    HIPCHK(hipGetLastError());
    c->d_Dtf.alloc(std::max<size_t>(c->d_Dt.n, 1));
    c->mixed_ready = true;
}

ShellMap shell_map(const eri_ctx *c)
{
    ShellMap m;
    m.shell_of_cart = c->d_soc.p;
    m.shell_of_sph = c->d_sos.p;
    m.l = c->d_l.p;
    m.cart_off = c->d_coff.p;
    m.sph_off = c->d_soff.p;
    return m;
}

bool ctx_ok(const eri_ctx *c) { return c && c->magic == 0x4d444a4b; }

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free build (build_jk_static): the Cartesian
// density and accumulators and the Hermite density / Hermite J of one build,
// carved from a file-scope device array.  Each GPU holds its own copy; its
// address is looked up once per device (at eri_setup, with that device
// current) and kept, since the array's name is not a device address in host
// code.
// ---------------------------------------------------------------------------
constexpr size_t kScratchDoubles = size_t(8) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[kScratchDoubles];
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch array (the device must be current).
double *scratch_address(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) {
        set_err(ERI_ESTATE, "device %d outside the %d devices the scratch table covers", dev, kMaxDevices);
        throw HipError{ERI_ESTATE};
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = (double *)ptr;
    }
    return g_scratch_ptr[dev];
}

// Doubles of scratch one build of this context needs (each region rounded up
// to 256 bytes).
size_t scratch_need(const eri_ctx *c)
{
    auto r = [](size_t n) { return (n + 31) / 32 * 32; };
    const size_t nc2 = (size_t)c->nbf_cart * c->nbf_cart;
    return 3 * r(nc2) + 2 * r(c->d_Dt.n);
}

// Does this launch take the single-precision share (two launches, modes 1/2)?
bool j_split(const eri_ctx *c, int X, int Y)
{
    return c->opts.precision == ERI_MIXED_ALL || (c->opts.precision == ERI_MIXED && c->jsplit[X][Y]);
}
bool k_split(const eri_ctx *c, size_t wi)
{
    return c->opts.precision == ERI_MIXED_ALL || (c->opts.precision == ERI_MIXED && c->ksplit[wi]);
}

template <typename F>
void timed(eri_ctx *c, hipStream_t st, const std::string &name, int work, int idx, int part, F &&launch)
{
    if (!c->profile) {
        launch();
        return;
    }
    eri_ctx::Rec r{name, nullptr, nullptr, work, idx, part};
    HIPCHK(hipEventCreate(&r.a));
    HIPCHK(hipEventCreate(&r.b));
    HIPCHK(hipEventRecord(r.a, st));
    launch();
    HIPCHK(hipEventRecord(r.b, st));
    c->pending.push_back(r);
}

std::string cls_name(const char *k, int a, int b, int cc, int d)
{
    char buf[40];
    snprintf(buf, sizeof(buf), "%s(%d%d|%d%d)", k, a, b, cc, d);
    return buf;
}

JArgs j_args(const eri_ctx *c, int X, int Y, bool mixed)
{
    JArgs a{};
    a.pp = c->d_pp.p;
    a.owner = c->d_owner.p + c->pp_base[X];
    a.Qbra = c->d_Q.p + c->cp_base[X];
    a.pbase = c->pp_base[X];
    a.nbp = c->npp[X];
    a.ket = c->d_cp.p + c->cp_base[Y];
    a.Qket = c->d_Q.p + c->cp_base[Y];
    a.nket = c->ncp[Y];
    a.kchunk = c->kchunk[X][Y];
    a.Dt = c->wk.Dt + c->dt_off[Y];
    a.dt_base = c->pp_base[Y];
    a.Jh = c->wk.Jh + c->jh_off[X];
    a.boys = c->d_boys.p;
    a.tau = c->opts.schwarz_thresh;
    a.tau_prim = c->opts.prim_thresh;
    a.mode = 0;
    if (mixed) {
        a.Dtf = c->d_Dtf.p + c->dt_off[Y];
        a.tau_mix = c->opts.mixed_thresh;
    }
    if (mixed || c->tau_dens > 0.0) {
        a.QDket = c->d_QD.p + c->cp_base[Y];
        a.tau_dens = c->tau_dens;
    }
    a.om2 = c->opts.omega * c->opts.omega;
    return a;
}


// Hermite density of every ket class, Hermite J cleared.
void j_prologue(eri_ctx *c, bool mixed, hipStream_t st)
{
    const int nc = c->nbf_cart;
    for (int Y = 0; Y < kPairClasses; ++Y)
        timed(c, st, cls_name("hdens", kPairL[Y][0], kPairL[Y][1], 0, 0), -1, 0, 0, [&] {
            launch_hermite_density(kPairL[Y][0], kPairL[Y][1], c->d_cp.p + c->cp_base[Y], c->ncp[Y], c->d_pp.p,
                                   c->wk.Pc, nc, c->wk.Dt + c->dt_off[Y],
                                   mixed ? c->d_Dtf.p + c->dt_off[Y] : nullptr, c->pp_base[Y], st);
        });
    timed(c, st, "fill_zero", -1, 0, 0, [&] { launch_fill_zero(c->wk.Jh, (int64_t)c->d_Jh.n, st); });
}

// The J-engine launches of every (bra class, ket class).
void j_classes(eri_ctx *c, bool mixed, hipStream_t st)
{
    for (int X = 0; X < kPairClasses; ++X) {
        if (c->npp[X] == 0) continue;
        for (int Y = 0; Y < kPairClasses; ++Y) {
            if (c->ncp[Y] == 0) continue;
            const int lx = kPairL[X][0] + kPairL[X][1], ly = kPairL[Y][0] + kPairL[Y][1];
            const std::string nm = cls_name(lx + ly <= 5 ? "jeng_small" : (jeng_is_reg(lx, ly) ? "jeng_reg" : "jeng_wave"),
                                            kPairL[X][0], kPairL[X][1], kPairL[Y][0], kPairL[Y][1]);
            JArgs a = j_args(c, X, Y, mixed);
            const bool split = mixed && j_split(c, X, Y);
            for (int part = split ? 1 : 0; part <= (split ? 2 : 0); ++part) {
                a.mode = part;
                timed(c, st, part == 0 ? nm : nm + (part == 1 ? "/d" : "/s"), 1, X * kPairClasses + Y, part,
                      [&] { launch_jeng(lx, ly, a, part == 2, st); });
            }
        }
    }
}

// Hermite J to Cartesian J, added into the accumulator.
void j_epilogue(eri_ctx *c, hipStream_t st)
{
    const int nc = c->nbf_cart;
    for (int X = 0; X < kPairClasses; ++X)
        timed(c, st, cls_name("herm2cart", kPairL[X][0], kPairL[X][1], 0, 0), -1, 0, 0, [&] {
            launch_hermite_to_cart(kPairL[X][0], kPairL[X][1], c->d_cp.p + c->cp_base[X], c->ncp[X], c->d_pp.p,
                                   c->wk.Jh + c->jh_off[X], c->pp_base[X], c->wk.Jacc, nc, st);
        });
}

KArgs k_args(const eri_ctx *c, const eri_ctx::KWork &w, bool mixed)
{
    KArgs a{};
    const int v = c->kinv[&w - c->kwork.data()];
    a.inv = v;
    a.bra = c->d_kcp[v].p + c->cp_base[w.X];
    a.ket = c->d_kcp[v].p + c->cp_base[w.Y];
    a.rows = c->d_rows.p + w.roff;
    a.prefix = c->d_prefix.p + w.off;
    a.nwork = w.nwork;
    a.nrows = w.nrows;
    a.same = w.X == w.Y;
    a.pp = c->d_pp.p;
    a.boys = c->d_boys.p;
    a.D = c->wk.Pc;
    a.Kacc = c->wk.Kacc;
    a.ld = c->nbf_cart;
    a.tau_prim = c->opts.prim_thresh;
    a.eprod_bra = c->d_eprod.p + c->eprod_off[w.X];
    a.pbase_bra = c->pp_base[w.X];
    a.eprod_ket = c->d_eprod.p + c->eprod_off[w.Y];
    a.pbase_ket = c->pp_base[w.Y];
    a.mode = 0;
    a.grid_cap = c->kcap[&w - c->kwork.data()];
    a.om2 = c->opts.omega * c->opts.omega;
    if (mixed) {
        a.eprodf_bra = c->d_eprodf.p + c->eprod_off[w.X];
        a.eprodf_ket = c->d_eprodf.p + c->eprod_off[w.Y];
        a.tau_mix = c->opts.mixed_thresh;
    }
    if (mixed || c->tau_dens > 0.0) {  // density-weighted bounds of the quartets
        a.Qbra = c->d_kQ[v].p + c->cp_base[w.X];
        a.Qket = c->d_kQ[v].p + c->cp_base[w.Y];
        a.Pm = c->d_Pm.p;
        a.nsh = c->nshell;
        a.tau_dens = c->tau_dens;
    }
    return a;
}

KPArgs kp_args(const KArgs &a, const int4 *chunks)
{
    KPArgs p{};
    p.bra = a.bra;
    p.ket = a.ket;
    p.chunks = chunks;
    p.rows = a.rows;
    p.prefix = a.prefix;
    p.same = a.same;
    p.pp = a.pp;
    p.eprod_bra = a.eprod_bra;
    p.pbase_bra = a.pbase_bra;
    p.eprod_ket = a.eprod_ket;
    p.pbase_ket = a.pbase_ket;
    p.boys = a.boys;
    p.D = a.D;
    p.Kacc = a.Kacc;
    p.ld = a.ld;
    p.tau_prim = a.tau_prim;
    p.eprodf_bra = a.eprodf_bra;
    p.eprodf_ket = a.eprodf_ket;
    p.mode = a.mode;
    p.tau_mix = a.tau_mix;
    p.Qbra = a.Qbra;
    p.Qket = a.Qket;
    p.Pm = a.Pm;
    p.nsh = a.nsh;
    p.om2 = a.om2;
    p.tau_dens = a.tau_dens;
    p.inv = a.inv;
    return p;
}


void run_j(eri_ctx *c, bool mixed, hipStream_t st)
{
    j_prologue(c, mixed, st);
    j_classes(c, mixed, st);
    j_epilogue(c, st);
}

// Range-walking wave classes on stA, lane-per-quartet classes on stB,
// bra-shared classes on stC.
void run_k(eri_ctx *c, bool mixed, hipStream_t stA, hipStream_t stB, hipStream_t stC)
{
    for (const auto &w : c->kwork) {
        if (w.nwork == 0) continue;
        const int la = kPairL[w.X][0], lb = kPairL[w.X][1], lc = kPairL[w.Y][0], ld = kPairL[w.Y][1];
        const int wi = (int)(&w - c->kwork.data());
        KArgs a = k_args(c, w, mixed);
        const bool split = mixed && k_split(c, (size_t)wi);
        for (int part = split ? 1 : 0; part <= (split ? 2 : 0); ++part) {
            a.mode = part;
            const bool f32 = part == 2;
            const char *sfx = part == 0 ? "" : (part == 1 ? "/d" : "/s");
            bool ok = false;
            if (w.choff >= 0) {
                const KPArgs p = kp_args(a, c->d_chunks.p + w.choff);
                const int nch = w.nchunks;
                hipStream_t st = stC;
                timed(c, st, cls_name("kp", la, lb, lc, ld) + sfx, 0, wi, part, [&] {
                    ok = launch_k_pair_0(la, lb, lc, ld, p, nch, f32, st) || launch_k_pair_1(la, lb, lc, ld, p, nch, f32, st) ||
                         launch_k_pair_2(la, lb, lc, ld, p, nch, f32, st) || launch_k_pair_3(la, lb, lc, ld, p, nch, f32, st) ||
                         launch_k_pair_4(la, lb, lc, ld, p, nch, f32, st) || launch_k_pair_5(la, lb, lc, ld, p, nch, f32, st) ||
                         launch_k_pair_6(la, lb, lc, ld, p, nch, f32, st) || launch_k_pair_7(la, lb, lc, ld, p, nch, f32, st);
                });
            } else {
                hipStream_t st = is_k_small(la, lb, lc, ld) ? stB : stA;
                timed(c, st, cls_name("k", la, lb, lc, ld) + sfx, 0, wi, part, [&] {
                    ok = launch_k_small(la, lb, lc, ld, a, f32, st) || launch_k_wave_0(la, lb, lc, ld, a, f32, st) ||
                         launch_k_wave_1(la, lb, lc, ld, a, f32, st) || launch_k_wave_2(la, lb, lc, ld, a, f32, st) ||
                         launch_k_wave_3(la, lb, lc, ld, a, f32, st) || launch_k_wave_4(la, lb, lc, ld, a, f32, st) ||
                         launch_k_wave_5(la, lb, lc, ld, a, f32, st);
                });
            }
            if (!ok) {
                set_err(ERI_ESTATE, "no exchange kernel for class (%d%d|%d%d)", la, lb, lc, ld);
                throw HipError{ERI_ESTATE};
            }
        }
    }
}

// Single-precision share of the last mixed build (same tile rules as the
// kernels).  Synchronous.
void mixed_counts(const eri_ctx *c)
{
    if (c->mix_counts_ok) return;
    const size_t nk = c->kwork.size();
    const size_t n = 2 * (nk + kPairClasses * kPairClasses);
    DevBuf<unsigned long long> cnt;
    cnt.alloc(n);
    HIPCHK(hipMemsetAsync(cnt.p, 0, n * sizeof(unsigned long long), c->st));
    for (size_t wi = 0; wi < nk; ++wi) {
        const auto &w = c->kwork[wi];
        if (w.nwork == 0 || !k_split(c, wi)) continue;
        KArgs a = k_args(c, w, true);
        const int la = kPairL[w.X][0], lb = kPairL[w.X][1], lc = kPairL[w.Y][0], ld = kPairL[w.Y][1];
        const int kind = w.choff >= 0 ? 2 : (is_k_small(la, lb, lc, ld) ? 0 : 1);
        launch_k_count_mix(a, kind, w.choff >= 0 ? c->d_chunks.p + w.choff : nullptr, w.nchunks, cnt.p + 2 * wi,
                           c->st);
    }
    for (int X = 0; X < kPairClasses; ++X)
        for (int Y = 0; Y < kPairClasses; ++Y) {
            if (c->npp[X] == 0 || c->ncp[Y] == 0 || !j_split(c, X, Y)) continue;
            JArgs a = j_args(c, X, Y, true);
            const int lx = kPairL[X][0] + kPairL[X][1], ly = kPairL[Y][0] + kPairL[Y][1];
            const int per_bra = (lx + ly > 5 && !jeng_is_reg(lx, ly)) ? 1 : 0;
            launch_j_count_mix(a, per_bra, cnt.p + 2 * (nk + X * kPairClasses + Y), c->st);
        }
    HIPCHK(hipGetLastError());
    std::vector<unsigned long long> h(n);
    HIPCHK(hipStreamSynchronize(c->st));
    HIPCHK(hipMemcpy(h.data(), cnt.p, n * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    c->kmix.assign(nk, {0, 0});
    for (size_t wi = 0; wi < nk; ++wi) c->kmix[wi] = {(int64_t)h[2 * wi], (int64_t)h[2 * wi + 1]};
    for (int X = 0; X < kPairClasses; ++X)
        for (int Y = 0; Y < kPairClasses; ++Y)
            for (int k = 0; k < 2; ++k) c->jmix[X][Y][k] = (int64_t)h[2 * (nk + X * kPairClasses + Y) + k];
    c->mix_counts_ok = true;
}

// Primitive quartets and model FLOPs of one profiled launch.
void rec_work(const eri_ctx *c, const eri_ctx::Rec &r, int64_t &pq, double &flops)
{
    pq = 0;
    flops = 0.0;
    if (r.work == 0) {
        const auto &w = c->kwork[r.idx];
        const int la = kPairL[w.X][0], lb = kPairL[w.X][1], lc = kPairL[w.Y][0], ld = kPairL[w.Y][1];
        int64_t p = c->kprim[r.idx], nw = w.nwork;
        if (r.part != 0) {
            mixed_counts(c);
            const int64_t ps = c->kmix[r.idx][0], ns = c->kmix[r.idx][1];
            p = r.part == 2 ? ps : p - ps;
            nw = r.part == 2 ? ns : nw - ns;
        }
        pq = p;
        flops = (double)p * fl_k_prim(la, lb, lc, ld) + (double)nw * fl_k_digest(la, lb, lc, ld);
    } else if (r.work == 1) {
        const int X = r.idx / kPairClasses, Y = r.idx % kPairClasses;
        int64_t p = c->jprim[X][Y];
        if (r.part != 0) {
            mixed_counts(c);
            const int64_t ps = c->jmix[X][Y][0];
            p = r.part == 2 ? ps : p - ps;
        }
        pq = p;
        flops = (double)p * fl_j_prim(kPairL[X][0] + kPairL[X][1], kPairL[Y][0] + kPairL[Y][1]);
    } else if (r.work == 2 || r.work == 3) {  // potential: idx = X * 16 + order, part = charges
        const int X = r.idx / 16, L = r.idx % 16;
        pq = (int64_t)c->npp[X] * r.part;
        flops = (double)pq * (r.work == 2 ? fl_v(L) : fl_vg(L));
    }
}

constexpr int kKgRange = 4;      // quartets per range of the exchange-gradient kernel
constexpr int kGradChunks = 32;  // most ket chunks of a gradient J-engine launch
constexpr int kKgMaxBlocks = 2048;

// Hermite arrays of order la+lb+1 of every primitive pair and the per-pair
// centre terms: the Coulomb and the potential gradients.
void ensure_jh1(eri_ctx *c)
{
    if (c->jh1_ready) return;
    size_t o = 0;
    for (int X = 0; X < kPairClasses; ++X) {
        c->jh1_off[X] = o;
        o += (size_t)c->npp[X] * nherm(kPairL[X][0] + kPairL[X][1] + 1);
    }
    c->d_Jh1.alloc(std::max<size_t>(o, 1));
    c->d_pg.alloc(std::max<size_t>(6 * c->cp.size(), 1));
    c->jh1_ready = true;
}

void ensure_grad(eri_ctx *c)
{
    if (c->grad_ready) return;
    ensure_jh1(c);
    // per-chunk Hermite J of one gradient J-engine launch (at most kGradChunks
    // ket chunks), reduced in chunk order
    size_t part = 1;
    for (int X = 0; X < kPairClasses; ++X)
        for (int Y = 0; Y < kPairClasses; ++Y) {
            const int ncp = c->ncp[Y];
            int kc = std::max(c->kchunk[X][Y], (ncp + kGradChunks - 1) / kGradChunks);
            kc = std::max(kc, 1);
            c->gchunk[X][Y] = kc;
            const size_t nch = (size_t)((ncp + kc - 1) / kc);
            part = std::max(part, nch * (size_t)c->npp[X] * nherm(kPairL[X][0] + kPairL[X][1] + 1));
        }
    c->d_jhpart.alloc(part);
    c->kg_blocks.assign(c->kwork.size(), 0);
    c->kg_off.assign(c->kwork.size(), 0);
    c->kg_total = 0;
    for (size_t wi = 0; wi < c->kwork.size(); ++wi) {
        const auto &w = c->kwork[wi];
        // small classes: a lane per quartet (64 per workgroup step); others a
        // workgroup per kKgRange quartets
        const int per = kg_small_class(kPairL[w.X][0], kPairL[w.X][1], kPairL[w.Y][0], kPairL[w.Y][1]) ? 64 : kKgRange;
        const int64_t ranges = (w.nwork + per - 1) / per;
        c->kg_blocks[wi] = (int)std::min<int64_t>(ranges, kKgMaxBlocks);
        c->kg_off[wi] = c->kg_total;
        c->kg_total += c->kg_blocks[wi];
    }
    c->d_kpart.alloc(std::max<size_t>((size_t)c->kg_total * 3 * c->natom, 1));
    c->grad_ready = true;
}

// dE/dR at fixed P (P_cart already in d_Pc).
void run_grad(eri_ctx *c, double *grad)
{
    hipStream_t st = c->st;
    const int nc = c->nbf_cart;
    ensure_grad(c);
    // mixed precision: the J-engine launches take the FP32 share that
    // build_jk's J-engine launches take (every launch under ERI_MIXED_ALL,
    // the autotuner's choice under ERI_MIXED), with the same density-weighted
    // tile rule; raised bra orders above 6 and the exchange part stay FP64
    const int prec = c->opts.precision;
    const bool mixed = prec != ERI_FP64;
    if (mixed) {
        ensure_mixed(c);
        launch_density_bounds(c->wk.Pc, nc, c->d_l.p, c->d_coff.p, c->nshell, c->d_Pm.p, c->d_cp.p, c->d_Q.p,
                              (int)c->cp.size(), c->d_QD.p, st);
    }
    // The Coulomb part runs on one internal stream and the exchange classes
    // are spread over the context stream and two more (each class writes
    // partials of its own, reduced in a fixed order at the end, so the
    // result does not depend on the interleaving); joined back before the
    // reduction.  While profiling, everything stays on the context stream.
    const bool fork = !c->profile && !c->recording;
    const hipStream_t sJ = fork ? c->aux[0] : st;
    const hipStream_t sK[3] = {st, fork ? c->aux[1] : st, fork ? c->aux[2] : st};
    if (fork) {
        HIPCHK(hipEventRecord(c->ev_fork, st));
        for (const hipStream_t s : {c->aux[0], c->aux[1], c->aux[2]}) HIPCHK(hipStreamWaitEvent(s, c->ev_fork, 0));
    }
    // Coulomb: Hermite density, J-engine with the bra order raised by one
    for (int Y = 0; Y < kPairClasses; ++Y)
        launch_hermite_density(kPairL[Y][0], kPairL[Y][1], c->d_cp.p + c->cp_base[Y], c->ncp[Y], c->d_pp.p,
                               c->wk.Pc, nc, c->wk.Dt + c->dt_off[Y], mixed ? c->d_Dtf.p + c->dt_off[Y] : nullptr,
                               c->pp_base[Y], sJ);
    launch_fill_zero(c->d_Jh1.p, (int64_t)c->d_Jh1.n, sJ);
    for (int X = 0; X < kPairClasses; ++X) {
        if (c->npp[X] == 0) continue;
        for (int Y = 0; Y < kPairClasses; ++Y) {
            if (c->ncp[Y] == 0) continue;
            JArgs a = j_args(c, X, Y, mixed);
            // every ket chunk stores its sums; they are added to Jh1 in chunk
            // order (the FP64 share first), so repeated gradients are bitwise
            // identical
            a.kchunk = c->gchunk[X][Y];
            const int nch = (c->ncp[Y] + a.kchunk - 1) / a.kchunk;
            const int lx = kPairL[X][0] + kPairL[X][1] + 1, ly = kPairL[Y][0] + kPairL[Y][1];
            a.Jh = c->d_jhpart.p;
            a.jh_part = (int64_t)c->npp[X] * nherm(lx);
            const bool split = mixed && lx <= 6 && (prec == ERI_MIXED_ALL || c->jsplit[X][Y]);
            for (int part = split ? 1 : 0; part <= (split ? 2 : 0); ++part) {
                a.mode = part;
                timed(c, sJ,
                      cls_name("jeng_grad", kPairL[X][0], kPairL[X][1], kPairL[Y][0], kPairL[Y][1]) +
                          (part == 0 ? "" : (part == 1 ? "/d" : "/s")),
                      -1, 0, 0, [&] {
                          if (!launch_jeng(lx, ly, a, part == 2, sJ)) {
                              set_err(ERI_ESTATE, "no J-engine kernel for orders (%d,%d)", lx, ly);
                              throw HipError{ERI_ESTATE};
                          }
                          launch_jh_reduce(c->d_jhpart.p, nch, a.jh_part, c->d_Jh1.p + c->jh1_off[X], a.jh_part,
                                           sJ);
                      });
            }
        }
    }
    for (int X = 0; X < kPairClasses; ++X) {
        JGArgs g{};
        g.cp = c->d_cp.p + c->cp_base[X];
        g.ncp = c->ncp[X];
        g.pp = c->d_pp.p;
        g.Jh1 = c->d_Jh1.p + c->jh1_off[X];
        g.jh_base = c->pp_base[X];
        g.D = c->wk.Pc;
        g.ld = nc;
        g.pg = c->d_pg.p + 6 * (size_t)c->cp_base[X];
        timed(c, sJ, cls_name("jgrad", kPairL[X][0], kPairL[X][1], 0, 0), -1, 0, 0,
              [&] { launch_jgrad(kPairL[X][0], kPairL[X][1], g, sJ); });
    }
    // exchange: every canonical quartet, all four centres; each class goes,
    // in class order, to the stream with the least model work so far
    double load[3] = {0.0, 0.0, 0.0};
    for (size_t wi = 0; wi < c->kwork.size(); ++wi) {
        const auto &w = c->kwork[wi];
        if (w.nwork == 0) continue;
        int si = 0;
        for (int k = 1; k < 3; ++k)
            if (load[k] < load[si]) si = k;
        const hipStream_t sk = sK[si];
        KGArgs g{};
        g.k = k_args(c, w, false);
        g.partial = c->d_kpart.p + (size_t)c->kg_off[wi] * 3 * c->natom;
        g.natom = c->natom;
        const int la = kPairL[w.X][0], lb = kPairL[w.X][1], lc = kPairL[w.Y][0], ld = kPairL[w.Y][1];
        const int nb = c->kg_blocks[wi];
        bool ok = false;
        timed(c, sk, cls_name("kgrad", la, lb, lc, ld), -1, 0, 0, [&] {
            ok = launch_kg_0(la, lb, lc, ld, g, nb, sk) || launch_kg_1(la, lb, lc, ld, g, nb, sk) ||
                 launch_kg_2(la, lb, lc, ld, g, nb, sk) || launch_kg_3(la, lb, lc, ld, g, nb, sk);
        });
        if (!ok) {
            set_err(ERI_ESTATE, "no exchange-gradient kernel for class (%d%d|%d%d)", la, lb, lc, ld);
            throw HipError{ERI_ESTATE};
        }
        const double prim = wi < c->kprim.size() ? (double)c->kprim[wi] : (double)w.nwork;
        load[si] += prim * fl_k_prim(la, lb, lc, ld) + (double)w.nwork * fl_k_digest(la, lb, lc, ld);
    }
    if (fork) {
        for (int k = 0; k < 3; ++k) {
            HIPCHK(hipEventRecord(c->ev_join[k], c->aux[k]));
            HIPCHK(hipStreamWaitEvent(st, c->ev_join[k], 0));
        }
    }
    const size_t nred = (size_t)grad_reduce_chunks((int)c->cp.size(), c->kg_total) * 3 * c->natom;
    if (c->d_gred.n < nred) c->d_gred.alloc(nred);
    launch_grad_reduce(c->d_cp.p, (int)c->cp.size(), c->d_pg.p, c->d_kpart.p, c->kg_total, c->natom, grad,
                       c->d_gred.p, st);
}

// V = sum_C q_C (m|1/|r - C||n): Hermite potential of every primitive pair
// (order la+lb), the J-engine's Hermite-to-Cartesian step, one triangle of
// the accumulator (V = Acc + Acc^T), then the output basis.
constexpr int64_t kVPartDoubles = 8 << 20;  // most charge-split partials of one potential launch

// charge splits of each class's Hermite potential of order la+lb+extra, and
// the partial buffer they need
void potential_plan(eri_ctx *c, int nchg, int extra, int *ns)
{
    size_t need = 1;
    for (int X = 0; X < kPairClasses; ++X) {
        const int L = kPairL[X][0] + kPairL[X][1] + extra;
        ns[X] = potential_splits(c->npp[X], nchg, L, kVPartDoubles);
        if (ns[X] > 1) need = std::max(need, (size_t)ns[X] * c->npp[X] * nherm(L));
    }
    if (c->d_vpart.n < need) c->d_vpart.alloc(need);
}

void run_potential(eri_ctx *c, const double *chg, int nchg, double *V)
{
    hipStream_t st = c->st;
    const int nc = c->nbf_cart;
    int ns[kPairClasses];
    potential_plan(c, nchg, 0, ns);
    launch_fill_zero(c->wk.Jacc, (int64_t)nc * nc, st);
    for (int X = 0; X < kPairClasses; ++X) {
        if (c->npp[X] == 0) continue;
        const int la = kPairL[X][0], lb = kPairL[X][1];
        double *vh = c->wk.Jh + c->jh_off[X];
        timed(c, st, cls_name("vh", la, lb, 0, 0), 2, X * 16 + la + lb, nchg, [&] {
            if (!launch_vh(la + lb, c->d_pp.p, c->pp_base[X], c->npp[X], chg, nchg, c->d_boys.p, vh,
                           c->d_vpart.p, ns[X], st)) {
                set_err(ERI_ESTATE, "no potential kernel for order %d", la + lb);
                throw HipError{ERI_ESTATE};
            }
        });
        launch_hermite_to_cart(la, lb, c->d_cp.p + c->cp_base[X], c->ncp[X], c->d_pp.p, vh, c->pp_base[X],
                               c->wk.Jacc, nc, st);
    }
    launch_acc_to_out(c->wk.Jacc, nc, V, c->nbf, shell_map(c), c->opts.spherical, st);
}

// dE_V/dR at fixed P (P_cart already in wk.Pc).  Atoms: the Hermite potential
// of order la+lb+1 through the Coulomb gradient's pair-derivative kernel;
// charges: the Hermite density against R of order la+lb+1.
void run_potential_grad(eri_ctx *c, const double *chg, int nchg, double *gatom, double *gchg)
{
    hipStream_t st = c->st;
    const int nc = c->nbf_cart;
    if (gatom) {
        ensure_jh1(c);
        int ns[kPairClasses];
        potential_plan(c, nchg, 1, ns);
        for (int X = 0; X < kPairClasses; ++X) {
            if (c->npp[X] == 0) continue;
            const int la = kPairL[X][0], lb = kPairL[X][1];
            double *vh = c->d_Jh1.p + c->jh1_off[X];
            timed(c, st, cls_name("vh1", la, lb, 0, 0), 2, X * 16 + la + lb + 1, nchg, [&] {
                if (!launch_vh(la + lb + 1, c->d_pp.p, c->pp_base[X], c->npp[X], chg, nchg, c->d_boys.p, vh,
                               c->d_vpart.p, ns[X], st)) {
                    set_err(ERI_ESTATE, "no potential kernel for order %d", la + lb + 1);
                    throw HipError{ERI_ESTATE};
                }
            });
            JGArgs g{};
            g.cp = c->d_cp.p + c->cp_base[X];
            g.ncp = c->ncp[X];
            g.pp = c->d_pp.p;
            g.Jh1 = vh;
            g.jh_base = c->pp_base[X];
            g.D = c->wk.Pc;
            g.ld = nc;
            g.pg = c->d_pg.p + 6 * (size_t)c->cp_base[X];
            launch_jgrad(la, lb, g, st);
        }
        const size_t nred = (size_t)grad_reduce_chunks((int)c->cp.size(), 0) * 3 * c->natom;
        if (c->d_gred.n < nred) c->d_gred.alloc(nred);
        launch_grad_reduce(c->d_cp.p, (int)c->cp.size(), c->d_pg.p, nullptr, 0, c->natom, gatom, c->d_gred.p, st);
    }
    if (gchg && nchg > 0) {
        launch_fill_zero(gchg, 3 * (int64_t)nchg, st);
        // pair splits per class: enough workgroups (64 charges each) to fill
        // the chip, at least 16 pairs per split
        const int groups = (nchg + 63) / 64;
        const int nshare = std::max(1, std::min(64, (4096 + groups - 1) / groups));
        const size_t need = (size_t)nshare * 3 * nchg;
        if (c->d_vpart.n < need) c->d_vpart.alloc(need);
        for (int X = 0; X < kPairClasses; ++X) {
            if (c->npp[X] == 0) continue;
            const int la = kPairL[X][0], lb = kPairL[X][1];
            launch_hermite_density(la, lb, c->d_cp.p + c->cp_base[X], c->ncp[X], c->d_pp.p, c->wk.Pc, nc,
                                   c->wk.Dt + c->dt_off[X], nullptr, c->pp_base[X], st);
            const int ns = std::max(1, std::min(nshare, (c->npp[X] + 15) / 16));
            timed(c, st, cls_name("vgrad_chg", la, lb, 0, 0), 3, X * 16 + la + lb, nchg, [&] {
                if (!launch_vgrad_charge(la + lb, c->d_pp.p, c->pp_base[X], c->npp[X], c->wk.Dt + c->dt_off[X],
                                         chg, nchg, c->d_boys.p, c->d_vpart.p, ns, gchg, st)) {
                    set_err(ERI_ESTATE, "no charge-gradient kernel for order %d", la + lb);
                    throw HipError{ERI_ESTATE};
                }
            });
        }
    }
}

}  // namespace

extern "C" {

void eri_default_opts(eri_opts *o)
{
    if (!o) return;
    o->schwarz_thresh = 1e-11;
    o->prim_thresh = 1e-13;
    o->mixed_thresh = 1e-5;
    o->precision = ERI_FP64;
    o->spherical = 1;
    o->stream = nullptr;
    o->omega = 0.0;
}

int eri_setup(const eri_shell *shells, int32_t nshell, const eri_atom *atoms, int32_t natom,
              const eri_opts *opts, eri_ctx **out)
{
    g_err.clear();
    if (!out) return set_err(ERI_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(shells, nshell, atoms, natom, opts);
    if (rc) return rc;
    std::unique_ptr<eri_ctx> c(new (std::nothrow) eri_ctx);
    if (!c) return set_err(ERI_ENOMEM, "host allocation failed");
    if (opts) c->opts = *opts; else eri_default_opts(&c->opts);
    c->st = (hipStream_t)c->opts.stream;
    c->nshell = nshell;
    c->natom = natom;
    try {
        HIPCHK(hipGetDevice(&c->device));
        (void)scratch_address(c->device);  // once per device: the scratch array's address
        for (auto &x : c->aux) HIPCHK(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->ev_kzero, hipEventDisableTiming));
        for (auto &e : c->ev_join) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->d_boys.upload(boys_table());
        build_basis(c.get(), shells, atoms);
        build_pairs(c.get());
        HIPCHK(hipStreamSynchronize(c->st));
    } catch (const HipError &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        return set_err(ERI_ENOMEM, "host allocation failed");
    }
    *out = c.release();
    return ERI_OK;
}

int eri_nbf(const eri_ctx *ctx, int32_t *nbf)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!nbf) return set_err(ERI_EINVAL, "nbf is NULL");
    *nbf = ctx->nbf;
    return ERI_OK;
}

int eri_set_geometry(eri_ctx *ctx, const eri_atom *atoms)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!atoms) return set_err(ERI_EINVAL, "atoms is NULL");
    for (int i = 0; i < ctx->natom; ++i)
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(atoms[i].xyz[k])) return set_err(ERI_EINVAL, "atom %d coordinate not finite", i);
    try {
        for (int i = 0; i < ctx->natom; ++i)
            for (int k = 0; k < 3; ++k) ctx->xyz[3 * i + k] = atoms[i].xyz[k];
        build_pairs(ctx);
        HIPCHK(hipStreamSynchronize(ctx->st));
        ++ctx->gen;
    } catch (const HipError &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        return set_err(ERI_ENOMEM, "host allocation failed");
    }
    return ERI_OK;
}

int eri_set_precision(eri_ctx *ctx, int32_t precision, double mixed_thresh)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (precision != ERI_FP64 && precision != ERI_MIXED && precision != ERI_MIXED_ALL)
        return set_err(ERI_EINVAL, "unknown precision %d", precision);
    if (!(mixed_thresh >= 0.0)) return set_err(ERI_EINVAL, "negative mixed threshold");
    if (ctx->opts.precision != precision || ctx->opts.mixed_thresh != mixed_thresh) ++ctx->gen;
    ctx->opts.precision = precision;
    ctx->opts.mixed_thresh = mixed_thresh;
    return ERI_OK;
}

int eri_set_omega(eri_ctx *ctx, double omega)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!(omega >= 0.0) || !std::isfinite(omega))
        return set_err(ERI_EINVAL, "omega %g not non-negative and finite", omega);
    if (ctx->opts.omega != omega) ++ctx->gen;
    ctx->opts.omega = omega;
    return ERI_OK;
}

int eri_set_density_screen(eri_ctx *ctx, double tau)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!(tau >= 0.0) || !std::isfinite(tau)) return set_err(ERI_EINVAL, "density screen %g not non-negative", tau);
    ctx->tau_dens = tau;
    ++ctx->gen;
    return ERI_OK;
}

int eri_one_electron(eri_ctx *ctx, double *S, double *T)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!S && !T) return set_err(ERI_EINVAL, "S and T are both NULL");
    try {
        hipStream_t st = ctx->st;
        const int nc = ctx->nbf_cart;
        launch_fill_zero(ctx->wk.Jacc, (int64_t)nc * nc, st);
        launch_fill_zero(ctx->wk.Kacc, (int64_t)nc * nc, st);
        for (int X = 0; X < kPairClasses; ++X)
            launch_st_pair(kPairL[X][0], kPairL[X][1], ctx->d_cp.p + ctx->cp_base[X], ctx->ncp[X], ctx->d_pp.p,
                           ctx->wk.Jacc, ctx->wk.Kacc, nc, st);
        const ShellMap m = shell_map(ctx);
        if (S) launch_acc_to_out(ctx->wk.Jacc, nc, S, ctx->nbf, m, ctx->opts.spherical, st);
        if (T) launch_acc_to_out(ctx->wk.Kacc, nc, T, ctx->nbf, m, ctx->opts.spherical, st);
        HIPCHK(hipGetLastError());
    } catch (const HipError &e) {
        return e.code;
    }
    return ERI_OK;
}

int build_jk(eri_ctx *ctx, const double *P, double *J, double *K)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!P) return set_err(ERI_EINVAL, "P is NULL");
    try {
        hipStream_t st = ctx->st;
        const ShellMap m = shell_map(ctx);
        const int nc = ctx->nbf_cart;
        const bool mixed = ctx->opts.precision != ERI_FP64;
        launch_p_to_cart(P, ctx->nbf, ctx->wk.Pc, nc, m, ctx->opts.spherical, st);
        if (mixed) ensure_mixed(ctx);
        if (mixed || ctx->tau_dens > 0.0) {
            launch_density_bounds(ctx->wk.Pc, nc, ctx->d_l.p, ctx->d_coff.p, ctx->nshell, ctx->d_Pm.p, ctx->d_cp.p,
                                  ctx->d_Q.p, (int)ctx->cp.size(), ctx->d_QD.p, st);
        }
        ctx->built_mixed = mixed;
        ctx->mix_counts_ok = false;
        // J on its own stream, K split over the context stream (range-walking
        // kernels) and two more (lane-per-quartet and bra-shared kernels); all
        // accumulate with atomics, so the four run concurrently.
        // While profiling, everything stays on the context stream so that
        // each kernel's events bracket it alone.
        const bool fork = !ctx->profile && !ctx->recording;
        HIPCHK(hipEventRecord(ctx->ev_fork, st));
        if (J) {
            hipStream_t sJ = fork ? ctx->aux[0] : st;
            HIPCHK(hipStreamWaitEvent(sJ, ctx->ev_fork, 0));
            launch_fill_zero(ctx->wk.Jacc, (int64_t)nc * nc, sJ);
            run_j(ctx, mixed, sJ);
            launch_acc_to_out(ctx->wk.Jacc, nc, J, ctx->nbf, m, ctx->opts.spherical, sJ);
            HIPCHK(hipEventRecord(ctx->ev_join[0], sJ));
        }
        if (K) {
            hipStream_t sK = fork ? ctx->aux[1] : st;
            launch_fill_zero(ctx->wk.Kacc, (int64_t)nc * nc, st);
            HIPCHK(hipEventRecord(ctx->ev_kzero, st));
            HIPCHK(hipStreamWaitEvent(sK, ctx->ev_kzero, 0));
            hipStream_t sP = fork ? ctx->aux[2] : st;
            HIPCHK(hipStreamWaitEvent(sP, ctx->ev_kzero, 0));
            run_k(ctx, mixed, st, sK, sP);
            HIPCHK(hipEventRecord(ctx->ev_join[1], sK));
            HIPCHK(hipEventRecord(ctx->ev_join[2], sP));
            HIPCHK(hipStreamWaitEvent(st, ctx->ev_join[1], 0));
            HIPCHK(hipStreamWaitEvent(st, ctx->ev_join[2], 0));
            launch_acc_to_out(ctx->wk.Kacc, nc, K, ctx->nbf, m, ctx->opts.spherical, st);
        }
        if (J) HIPCHK(hipStreamWaitEvent(st, ctx->ev_join[0], 0));
        HIPCHK(hipGetLastError());
    } catch (const HipError &e) {
        return e.code;
    }
    return ERI_OK;
}

int build_jk_static(eri_ctx *ctx, const double *P, double *J, double *K)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!P) return set_err(ERI_EINVAL, "P is NULL");
    if (ctx->opts.precision != ERI_FP64)
        return set_err(ERI_ESTATE, "build_jk_static runs the double-precision path only (precision %d)",
                       ctx->opts.precision);
    const size_t need = scratch_need(ctx);
    if (need > kScratchDoubles)
        return set_err(ERI_EINVAL, "build_jk_static: this context needs %zu bytes of scratch, more than the "
                                   "%zu-byte static array (nbf_cart %d)",
                       need * sizeof(double), kScratchDoubles * sizeof(double), ctx->nbf_cart);
    double *base = nullptr;
    try {
        base = scratch_address(ctx->device);
    } catch (const HipError &e) {
        return e.code;
    }
    auto r = [](size_t n) { return (n + 31) / 32 * 32; };
    const size_t nc2 = (size_t)ctx->nbf_cart * ctx->nbf_cart;
    const eri_ctx::Work own = ctx->wk;
    ctx->wk.Pc = base;
    ctx->wk.Jacc = base + r(nc2);
    ctx->wk.Kacc = base + 2 * r(nc2);
    ctx->wk.Dt = base + 3 * r(nc2);
    ctx->wk.Jh = base + 3 * r(nc2) + r(ctx->d_Dt.n);
    const int rc = build_jk(ctx, P, J, K);
    ctx->wk = own;
    return rc;
}

int jk_grad(eri_ctx *ctx, const double *P, double *grad, double *E)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!P) return set_err(ERI_EINVAL, "P is NULL");
    if (!grad && !E) return set_err(ERI_EINVAL, "grad and E are both NULL");
    try {
        hipStream_t st = ctx->st;
        const ShellMap m = shell_map(ctx);
        if (E) {
            const size_t n2 = (size_t)ctx->nbf * ctx->nbf;
            if (ctx->d_Jtmp.n != n2) {
                ctx->d_Jtmp.alloc(n2);
                ctx->d_Ktmp.alloc(n2);
            }
            const int32_t prec = ctx->opts.precision;
            ctx->opts.precision = ERI_FP64;
            const int rc = build_jk(ctx, P, ctx->d_Jtmp.p, ctx->d_Ktmp.p);
            ctx->opts.precision = prec;
            if (rc) return rc;
            launch_energy(P, ctx->d_Jtmp.p, ctx->d_Ktmp.p, (int64_t)n2, E, st);
        }
        if (grad) {
            launch_p_to_cart(P, ctx->nbf, ctx->wk.Pc, ctx->nbf_cart, m, ctx->opts.spherical, st);
            run_grad(ctx, grad);
        }
        HIPCHK(hipGetLastError());
    } catch (const HipError &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        return set_err(ERI_ENOMEM, "host allocation failed");
    }
    return ERI_OK;
}

// Bounding sphere of every contracted pair: all points where one of its
// primitives has p |r - P|^2 <= kGridCut.
void ensure_grid(eri_ctx *c)
{
    if (c->grid_ready) return;
    std::vector<double4> sph(std::max<size_t>(c->cp.size(), 1));
    for (size_t k = 0; k < c->cp.size(); ++k) {
        const CPair &A = c->cp[k];
        double cx = 0.0, cy = 0.0, cz = 0.0;
        for (int i = 0; i < A.np; ++i) {
            const PrimPair &q = c->pp[A.poff + i];
            cx += q.P[0];
            cy += q.P[1];
            cz += q.P[2];
        }
        cx /= A.np;
        cy /= A.np;
        cz /= A.np;
        double r = 0.0;
        for (int i = 0; i < A.np; ++i) {
            const PrimPair &q = c->pp[A.poff + i];
            const double d = std::sqrt((q.P[0] - cx) * (q.P[0] - cx) + (q.P[1] - cy) * (q.P[1] - cy) +
                                       (q.P[2] - cz) * (q.P[2] - cz));
            r = std::max(r, d + std::sqrt(kGridCut / q.p));
        }
        sph[k] = make_double4(cx, cy, cz, r * (1.0 + 1e-12) + 1e-12);
    }
    c->d_psph.upload(sph);
    c->d_xyz.upload(c->xyz);
    c->grid_ready = true;
}

void grid_prepare(eri_ctx *c, const double *pts, int64_t npts)
{
    ensure_grid(c);
    const size_t nblk = (size_t)((npts + 63) / 64);
    if (c->d_bsph.n < nblk) c->d_bsph.alloc(nblk);
    launch_grid_blocks(pts, npts, c->d_bsph.p, c->st);
}

int eri_potential(eri_ctx *ctx, const double *charges, int32_t ncharge, double *V)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!V) return set_err(ERI_EINVAL, "V is NULL");
    if (ncharge < 0) return set_err(ERI_EINVAL, "ncharge %d negative", ncharge);
    if (ncharge > 0 && !charges) return set_err(ERI_EINVAL, "charges is NULL");
    try {
        run_potential(ctx, charges, ncharge, V);
        HIPCHK(hipGetLastError());
    } catch (const HipError &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        return set_err(ERI_ENOMEM, "host allocation failed");
    }
    return ERI_OK;
}

int eri_potential_grad(eri_ctx *ctx, const double *charges, int32_t ncharge, const double *P, double *gatom,
                       double *gchg)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!P) return set_err(ERI_EINVAL, "P is NULL");
    if (!gatom && !gchg) return set_err(ERI_EINVAL, "gatom and gchg are both NULL");
    if (ncharge < 0) return set_err(ERI_EINVAL, "ncharge %d negative", ncharge);
    if (ncharge > 0 && !charges) return set_err(ERI_EINVAL, "charges is NULL");
    try {
        launch_p_to_cart(P, ctx->nbf, ctx->wk.Pc, ctx->nbf_cart, shell_map(ctx), ctx->opts.spherical, ctx->st);
        run_potential_grad(ctx, charges, ncharge, gatom, gchg);
        HIPCHK(hipGetLastError());
    } catch (const HipError &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        return set_err(ERI_ENOMEM, "host allocation failed");
    }
    return ERI_OK;
}

int eri_grid_density(eri_ctx *ctx, const double *P, const double *pts, int64_t npts, double *rho, double *grad)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!P) return set_err(ERI_EINVAL, "P is NULL");
    if (npts < 0) return set_err(ERI_EINVAL, "npts %lld negative", (long long)npts);
    if (npts == 0) return ERI_OK;
    if (!pts || !rho) return set_err(ERI_EINVAL, "pts or rho is NULL");
    try {
        hipStream_t st = ctx->st;
        const int nc = ctx->nbf_cart;
        launch_p_to_cart(P, ctx->nbf, ctx->wk.Pc, nc, shell_map(ctx), ctx->opts.spherical, st);
        grid_prepare(ctx, pts, npts);
        launch_fill_zero(rho, npts, st);
        if (grad) launch_fill_zero(grad, 3 * npts, st);
        // The pair classes add into the points class by class.  They run on
        // the context stream (into rho, grad) and three internal ones (each
        // into a zeroed partial of its own), each class to the stream with
        // the least pair work so far; after the join the partials are added
        // in stream order, so the result is reproducible bit for bit.  Not
        // forked while profiling, or when the partials would pass 1 GiB.
        const int64_t w = grad ? 4 : 1;  // doubles per point
        const bool fork = !ctx->profile && !ctx->recording && 3 * w * npts * (int64_t)sizeof(double) <= (1ll << 30);
        double *part = nullptr;
        if (fork) {
            if (ctx->d_gpart.n < (size_t)(3 * w * npts)) ctx->d_gpart.alloc((size_t)(3 * w * npts));
            part = ctx->d_gpart.p;
            launch_fill_zero(part, 3 * w * npts, st);
            HIPCHK(hipEventRecord(ctx->ev_fork, st));
            for (int k = 0; k < 3; ++k) HIPCHK(hipStreamWaitEvent(ctx->aux[k], ctx->ev_fork, 0));
        }
        double load[4] = {0.0, 0.0, 0.0, 0.0};
        for (int X = 0; X < kPairClasses; ++X) {
            if (ctx->ncp[X] == 0) continue;
            int si = 0;
            if (fork)
                for (int k = 1; k < 4; ++k)
                    if (load[k] < load[si]) si = k;
            load[si] += (double)ctx->ncp[X] * ncart(kPairL[X][0]) * ncart(kPairL[X][1]);
            const hipStream_t sg = si == 0 ? st : ctx->aux[si - 1];
            double *r = si == 0 ? rho : part + (int64_t)(si - 1) * npts;
            double *g = !grad ? nullptr : (si == 0 ? grad : part + 3 * npts + (int64_t)(si - 1) * 3 * npts);
            timed(ctx, sg, cls_name("grid_rho", kPairL[X][0], kPairL[X][1], 0, 0), -1, 0, 0, [&] {
                launch_grid_rho(kPairL[X][0], kPairL[X][1], ctx->d_cp.p + ctx->cp_base[X], ctx->ncp[X], ctx->d_pp.p,
                                ctx->d_psph.p + ctx->cp_base[X], ctx->d_xyz.p, ctx->wk.Pc, nc, pts, npts,
                                ctx->d_bsph.p, r, g, sg);
            });
        }
        if (fork) {
            for (int k = 0; k < 3; ++k) {
                HIPCHK(hipEventRecord(ctx->ev_join[k], ctx->aux[k]));
                HIPCHK(hipStreamWaitEvent(st, ctx->ev_join[k], 0));
            }
            launch_jh_reduce(part, 3, npts, rho, npts, st);
            if (grad) launch_jh_reduce(part + 3 * npts, 3, 3 * npts, grad, 3 * npts, st);
        }
        HIPCHK(hipGetLastError());
    } catch (const HipError &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        return set_err(ERI_ENOMEM, "host allocation failed");
    }
    return ERI_OK;
}

int eri_grid_matrix(eri_ctx *ctx, const double *pts, int64_t npts, const double *v0, const double *v1, double *V)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!V) return set_err(ERI_EINVAL, "V is NULL");
    if (npts < 0) return set_err(ERI_EINVAL, "npts %lld negative", (long long)npts);
    if (npts > 0 && (!pts || !v0)) return set_err(ERI_EINVAL, "pts or v0 is NULL");
    try {
        hipStream_t st = ctx->st;
        const int nc = ctx->nbf_cart;
        launch_fill_zero(ctx->wk.Jacc, (int64_t)nc * nc, st);
        if (npts > 0) {
            grid_prepare(ctx, pts, npts);
            // every contracted pair stores its own block, so the pair classes
            // run concurrently on the context stream and three internal ones
            // (each class to the stream with the least pair-block work so
            // far), joined back before the output transform; while
            // profiling, everything stays on the context stream
            const bool fork = !ctx->profile && !ctx->recording;
            const hipStream_t ss[4] = {st, fork ? ctx->aux[0] : st, fork ? ctx->aux[1] : st,
                                       fork ? ctx->aux[2] : st};
            if (fork) {
                HIPCHK(hipEventRecord(ctx->ev_fork, st));
                for (int k = 0; k < 3; ++k) HIPCHK(hipStreamWaitEvent(ctx->aux[k], ctx->ev_fork, 0));
            }
            double load[4] = {0.0, 0.0, 0.0, 0.0};
            for (int X = 0; X < kPairClasses; ++X) {
                if (ctx->ncp[X] == 0) continue;
                int si = 0;
                for (int k = 1; k < 4; ++k)
                    if (load[k] < load[si]) si = k;
                const hipStream_t sg = ss[si];
                load[si] += (double)ctx->ncp[X] * ncart(kPairL[X][0]) * ncart(kPairL[X][1]);
                timed(ctx, sg, cls_name("grid_vmat", kPairL[X][0], kPairL[X][1], 0, 0), -1, 0, 0, [&] {
                    launch_grid_vmat(kPairL[X][0], kPairL[X][1], ctx->d_cp.p + ctx->cp_base[X], ctx->ncp[X],
                                     ctx->d_pp.p, ctx->d_psph.p + ctx->cp_base[X], ctx->d_xyz.p, pts, npts,
                                     ctx->d_bsph.p, v0, v1, ctx->wk.Jacc, nc, sg);
                });
            }
            if (fork) {
                for (int k = 0; k < 3; ++k) {
                    HIPCHK(hipEventRecord(ctx->ev_join[k], ctx->aux[k]));
                    HIPCHK(hipStreamWaitEvent(st, ctx->ev_join[k], 0));
                }
            }
        }
        launch_acc_to_out(ctx->wk.Jacc, nc, V, ctx->nbf, shell_map(ctx), ctx->opts.spherical, st);
        HIPCHK(hipGetLastError());
    } catch (const HipError &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        return set_err(ERI_ENOMEM, "host allocation failed");
    }
    return ERI_OK;
}

int eri_energy(eri_ctx *ctx, const double *P, const double *J, const double *K, double *E)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!P || !J || !K || !E) return set_err(ERI_EINVAL, "null argument");
    try {
        launch_energy(P, J, K, (int64_t)ctx->nbf * ctx->nbf, E, ctx->st);
        HIPCHK(hipGetLastError());
    } catch (const HipError &e) {
        return e.code;
    }
    return ERI_OK;
}

int eri_stats(const eri_ctx *ctx, eri_stats_t *out)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!out) return set_err(ERI_EINVAL, "out is NULL");
    memset(out, 0, sizeof(*out));
    out->nshell = ctx->nshell;
    out->natom = ctx->natom;
    out->nbf = ctx->nbf;
    out->nbf_cart = ctx->nbf_cart;
    out->n_pairs = (int64_t)ctx->cp.size();
    out->n_prim_pairs = (int64_t)ctx->pp.size();
    out->n_quartets = ctx->n_quartets;
    if (ctx->built_mixed) {
        try {
            mixed_counts(ctx);
        } catch (const HipError &e) {
            return e.code;
        }
        for (const auto &v : ctx->kmix) out->n_quartets_fp32 += v[1];
    }
    out->eris_sph = ctx->eris_sph;
    out->eris_cart = ctx->eris_cart;
    out->model_flops_k = ctx->model_flops_k;
    out->model_flops_j = ctx->model_flops_j;
    out->last_ms = ctx->last_ms;
    for (int64_t v : ctx->kprim) out->n_prim_quartets_k += v;
    for (int X = 0; X < kPairClasses; ++X)
        for (int Y = 0; Y < kPairClasses; ++Y) out->n_prim_quartets_j += ctx->jprim[X][Y];
    return ERI_OK;
}

int eri_set_profiling(eri_ctx *ctx, int32_t on)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    ctx->profile = on != 0;
    return ERI_OK;
}

int eri_profile_read(eri_ctx *ctx, eri_kernel_time *out, int32_t cap, int32_t *n)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!n || (cap > 0 && !out)) return set_err(ERI_EINVAL, "null output");
    try {
        HIPCHK(hipStreamSynchronize(ctx->st));
        for (auto &x : ctx->aux) HIPCHK(hipStreamSynchronize(x));
        for (auto &r : ctx->pending) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
            auto &acc = ctx->prof[r.name];
            acc.launches += 1;
            acc.ms += ms;
            rec_work(ctx, r, acc.pq, acc.flops);
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        ctx->pending.clear();
    } catch (const HipError &e) {
        return e.code;
    }
    int k = 0;
    for (auto &kv : ctx->prof) {
        if (k < cap) {
            memset(&out[k], 0, sizeof(eri_kernel_time));
            snprintf(out[k].name, sizeof(out[k].name), "%s", kv.first.c_str());
            out[k].launches = kv.second.launches;
            out[k].ms = kv.second.ms;
            out[k].flops = kv.second.flops;
            out[k].prim_quartets = kv.second.pq;
        }
        ++k;
    }
    *n = k;
    ctx->prof.clear();
    return ERI_OK;
}

int eri_destroy(eri_ctx *ctx)
{
    if (!ctx) return ERI_OK;
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (ctx->st) (void)hipStreamSynchronize(ctx->st); else (void)hipDeviceSynchronize();
    for (auto &x : ctx->aux)
        if (x) {
            (void)hipStreamSynchronize(x);
            (void)hipStreamDestroy(x);
        }
    for (hipEvent_t e : {ctx->ev_fork, ctx->ev_kzero, ctx->ev_join[0], ctx->ev_join[1], ctx->ev_join[2]})
        if (e) (void)hipEventDestroy(e);
    for (auto &r : ctx->pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    ctx->magic = 0;
    delete ctx;
    return ERI_OK;
}

const char *eri_last_error(void) { return g_err.c_str(); }

/* Autotuner: times the candidate launch shapes of every J-engine and
 * range-walking exchange launch on this context's own workload (density P,
 * current precision) and keeps the fastest. */
int eri_autotune(eri_ctx *ctx, const double *P, int32_t reps)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!P) return set_err(ERI_EINVAL, "P is NULL");
    if (reps < 1) reps = 1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool prof = ctx->profile;
    ctx->profile = false;
    try {
        const size_t n2 = (size_t)ctx->nbf * ctx->nbf;
        if (ctx->d_Jtmp.n != n2) {
            ctx->d_Jtmp.alloc(n2);
            ctx->d_Ktmp.alloc(n2);
        }
        int rc = build_jk(ctx, P, ctx->d_Jtmp.p, ctx->d_Ktmp.p);  // P_cart, bounds, Hermite density
        if (rc) {
            ctx->profile = prof;
            return rc;
        }
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        hipStream_t st = ctx->st;
        const bool mixed = ctx->opts.precision != ERI_FP64;
        auto time_it = [&](auto &&launch) {
            float best = 1e30f;
            for (int r = 0; r < reps; ++r) {
                HIPCHK(hipEventRecord(e0, st));
                launch();
                HIPCHK(hipEventRecord(e1, st));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                best = std::min(best, ms);
            }
            return best;
        };
        // split options: ERI_MIXED tries both (the FP32 share is kept only
        // where it is faster); ERI_MIXED_ALL and ERI_FP64 have one
        const int prec = ctx->opts.precision;
        const bool tune_split = prec == ERI_MIXED;
        static const int kChunks[] = {8, 16, 32, 64, 128, 256, 512, 1024};
        for (int X = 0; X < kPairClasses; ++X)
            for (int Y = 0; Y < kPairClasses; ++Y) {
                if (ctx->npp[X] == 0 || ctx->ncp[Y] == 0) continue;
                const int lx = kPairL[X][0] + kPairL[X][1], ly = kPairL[Y][0] + kPairL[Y][1];
                float best = 1e30f;
                int pick = ctx->kchunk[X][Y];
                bool pick_split = ctx->jsplit[X][Y];
                for (int sp = 0; sp < 2; ++sp) {
                    const bool split = tune_split ? sp == 1 : (sp == 0 && prec == ERI_MIXED_ALL);
                    if (!tune_split && sp == 1) break;
                    for (int kc : kChunks) {
                        JArgs a = j_args(ctx, X, Y, mixed);
                        a.kchunk = kc;
                        const float ms = time_it([&] {
                            for (int part = split ? 1 : 0; part <= (split ? 2 : 0); ++part) {
                                a.mode = part;
                                launch_jeng(lx, ly, a, part == 2, st);
                            }
                        });
                        if (ms < best) {
                            best = ms;
                            pick = kc;
                            pick_split = split;
                        }
                    }
                }
                ctx->kchunk[X][Y] = pick;
                if (tune_split) ctx->jsplit[X][Y] = pick_split;
            }
        // one exchange launch as build_jk runs it (its current split choice)
        auto launch_k = [&](const eri_ctx::KWork &w, KArgs a, bool split) {
            const int la = kPairL[w.X][0], lb = kPairL[w.X][1], lc = kPairL[w.Y][0], ld = kPairL[w.Y][1];
            for (int part = split ? 1 : 0; part <= (split ? 2 : 0); ++part) {
                a.mode = part;
                const bool f32 = part == 2;
                if (w.choff >= 0) {
                    const KPArgs kp = kp_args(a, ctx->d_chunks.p + w.choff);
                    (void)(launch_k_pair_0(la, lb, lc, ld, kp, w.nchunks, f32, st) ||
                           launch_k_pair_1(la, lb, lc, ld, kp, w.nchunks, f32, st) ||
                           launch_k_pair_2(la, lb, lc, ld, kp, w.nchunks, f32, st) ||
                           launch_k_pair_3(la, lb, lc, ld, kp, w.nchunks, f32, st) ||
                           launch_k_pair_4(la, lb, lc, ld, kp, w.nchunks, f32, st) ||
                           launch_k_pair_5(la, lb, lc, ld, kp, w.nchunks, f32, st) ||
                           launch_k_pair_6(la, lb, lc, ld, kp, w.nchunks, f32, st) ||
                           launch_k_pair_7(la, lb, lc, ld, kp, w.nchunks, f32, st));
                } else {
                    (void)(launch_k_small(la, lb, lc, ld, a, f32, st) ||
                           launch_k_wave_0(la, lb, lc, ld, a, f32, st) || launch_k_wave_1(la, lb, lc, ld, a, f32, st) ||
                           launch_k_wave_2(la, lb, lc, ld, a, f32, st) || launch_k_wave_3(la, lb, lc, ld, a, f32, st) ||
                           launch_k_wave_4(la, lb, lc, ld, a, f32, st) || launch_k_wave_5(la, lb, lc, ld, a, f32, st));
                }
            }
        };
        // exchange variant of every lane-per-item launch: kets grouped by
        // their first shell (view 0) or by their second (view 1, the paper's
        // inverted ordering), whichever is faster on this workload
        {
            const size_t nw = ctx->kwork.size();
            std::vector<float> tv[2];
            HIPCHK(hipStreamSynchronize(st));
            for (int v = 0; v < 2; ++v) {
                for (size_t wi = 0; wi < nw; ++wi) ctx->kinv[wi] = v;
                build_kwork(ctx);
                tv[v].assign(nw, 1e30f);
                for (size_t wi = 0; wi < nw; ++wi) {
                    const auto &w = ctx->kwork[wi];
                    if (w.nwork == 0 || !kinv_ok(w.X, w.Y)) continue;
                    const KArgs a = k_args(ctx, w, mixed);
                    const bool split = mixed && (prec == ERI_MIXED_ALL || ctx->ksplit[wi]);
                    tv[v][wi] = time_it([&] { launch_k(w, a, split); });
                }
            }
            for (size_t wi = 0; wi < nw; ++wi) ctx->kinv[wi] = tv[1][wi] < tv[0][wi] ? 1 : 0;
            build_kwork(ctx);
        }
        static const int kCaps[] = {1024, 4096, 16384, 32768, 131072};
        for (size_t wi = 0; wi < ctx->kwork.size(); ++wi) {
            const auto &w = ctx->kwork[wi];
            const int la = kPairL[w.X][0], lb = kPairL[w.X][1], lc = kPairL[w.Y][0], ld = kPairL[w.Y][1];
            if (w.nwork == 0) continue;
            const bool wave = w.choff < 0 && !is_k_small(la, lb, lc, ld);
            if (!wave && !tune_split) continue;
            float best = 1e30f;
            int pick = ctx->kcap[wi];
            bool pick_split = ctx->ksplit[wi] != 0;
            for (int sp = 0; sp < 2; ++sp) {
                const bool split = tune_split ? sp == 1 : (sp == 0 && prec == ERI_MIXED_ALL);
                if (!tune_split && sp == 1) break;
                for (int cap : kCaps) {
                    if (!wave && cap != kCaps[0]) break;  // only the split choice for these
                    KArgs a = k_args(ctx, w, mixed);
                    a.grid_cap = wave ? cap : 0;
                    const float ms = time_it([&] { launch_k(w, a, split); });
                    if (ms < best) {
                        best = ms;
                        pick = wave ? cap : 0;
                        pick_split = split;
                    }
                }
            }
            ctx->kcap[wi] = pick;
            if (tune_split) ctx->ksplit[wi] = pick_split;
        }
        ++ctx->gen;
    } catch (const HipError &e) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        ctx->profile = prof;
        return e.code;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->profile = prof;
    return ERI_OK;
}

/* Current launch-shape choice (for reports): J-engine ket chunk of (X, Y)
 * and the exchange workgroup cap of launch wi (0 = default). */
int eri_tuning(const eri_ctx *ctx, int32_t *kchunk100, int32_t *kcap, int32_t cap_len, int32_t *n_kcap)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (kchunk100)
        for (int X = 0; X < kPairClasses; ++X)
            for (int Y = 0; Y < kPairClasses; ++Y) kchunk100[X * kPairClasses + Y] = ctx->kchunk[X][Y];
    if (n_kcap) *n_kcap = (int32_t)ctx->kcap.size();
    if (kcap)
        for (int32_t i = 0; i < cap_len && i < (int32_t)ctx->kcap.size(); ++i) kcap[i] = ctx->kcap[i];
    return ERI_OK;
}

int eri_get_tuning(const eri_ctx *ctx, eri_tuning_t *out)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!out) return set_err(ERI_EINVAL, "out is NULL");
    memset(out, 0, sizeof(*out));
    for (int X = 0; X < kPairClasses; ++X)
        for (int Y = 0; Y < kPairClasses; ++Y) {
            out->kchunk[X * kPairClasses + Y] = ctx->kchunk[X][Y];
            out->jsplit[X * kPairClasses + Y] = ctx->jsplit[X][Y] ? 1 : 0;
        }
    const int nk = (int)std::min<size_t>(ctx->kwork.size(), 64);
    out->n_kwork = nk;
    for (int i = 0; i < nk; ++i) {
        out->kwork_class[i] = ctx->kwork[i].X * kPairClasses + ctx->kwork[i].Y;
        out->kcap[i] = ctx->kcap[i];
        out->ksplit[i] = ctx->ksplit[i] ? 1 : 0;
        out->kinv[i] = ctx->kinv[i];
    }
    return ERI_OK;
}

int eri_set_tuning(eri_ctx *ctx, const eri_tuning_t *in)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (!in) return set_err(ERI_EINVAL, "in is NULL");
    for (int k = 0; k < kPairClasses * kPairClasses; ++k)
        if (in->kchunk[k] < 8 || in->kchunk[k] > 1024)
            return set_err(ERI_EINVAL, "kchunk[%d] = %d outside 8..1024", k, in->kchunk[k]);
    if (in->n_kwork < 0 || in->n_kwork > 64) return set_err(ERI_EINVAL, "n_kwork %d outside 0..64", in->n_kwork);
    for (int i = 0; i < in->n_kwork; ++i) {
        if (in->kcap[i] < 0) return set_err(ERI_EINVAL, "kcap[%d] = %d negative", i, in->kcap[i]);
        if (in->kinv[i] != 0 && in->kinv[i] != 1) return set_err(ERI_EINVAL, "kinv[%d] = %d not 0 or 1", i, in->kinv[i]);
    }
    for (int X = 0; X < kPairClasses; ++X)
        for (int Y = 0; Y < kPairClasses; ++Y) {
            ctx->kchunk[X][Y] = in->kchunk[X * kPairClasses + Y];
            ctx->jsplit[X][Y] = in->jsplit[X * kPairClasses + Y] != 0;
        }
    bool views_changed = false;
    for (size_t wi = 0; wi < ctx->kwork.size(); ++wi) {
        const int cls = ctx->kwork[wi].X * kPairClasses + ctx->kwork[wi].Y;
        for (int i = 0; i < in->n_kwork; ++i)
            if (in->kwork_class[i] == cls) {
                ctx->kcap[wi] = in->kcap[i];
                ctx->ksplit[wi] = in->ksplit[i] != 0;
                const int v = in->kinv[i] && kinv_ok(ctx->kwork[wi].X, ctx->kwork[wi].Y) ? 1 : 0;
                views_changed |= v != ctx->kinv[wi];
                ctx->kinv[wi] = v;
            }
    }
    if (views_changed) {
        try {
            HIPCHK(hipStreamSynchronize(ctx->st));  // the old lists may still be read
            build_kwork(ctx);
        } catch (const HipError &e) {
            return e.code;
        } catch (const std::bad_alloc &) {
            return set_err(ERI_ENOMEM, "host allocation failed");
        }
    }
    ctx->mix_counts_ok = false;
    ++ctx->gen;
    return ERI_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: the J/K builds of many contexts recorded once into a HIP graph.
// Each molecule is a branch forked from the batch stream onto one of a few
// streams and joined back, so independent molecules overlap on the device
// and a whole batch costs one graph launch.  The graph is recorded on the
// first build and again whenever the pointers or a context change.
// ---------------------------------------------------------------------------
struct eri_batch {
    uint32_t magic = 0x4d4a4b42;
    std::vector<eri_ctx *> ctxs;
    std::vector<uint64_t> gens;
    hipStream_t st = nullptr;      // caller's stream (graph launches)
    std::vector<hipStream_t> lanes;  // branch streams used while recording
    std::vector<hipEvent_t> evs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const double *> P;
    std::vector<double *> J, K;
    // direct launches: issue order (largest first) and lane of every molecule,
    // timing events of the last call (start, then one per molecule)
    std::vector<int> order, lane_of;
    std::vector<hipEvent_t> tev;
    bool timed_once = false;
    // queue launches (double-precision batches): one persistent launch per
    // kernel instantiation over the blocks of every molecule
    struct QGroup {
        QueueLaunchFn fn;
        const char *kind;
        size_t tab_off;   // bytes into d_qtab
        size_t item_off;  // into d_qitems
        int nitems, entries;
    };
    int32_t mode = ERI_BATCH_QUEUE;
    // queue builds fork from the batch stream as build_jk does: J-engine
    // launches on qaux[0], lane-per-quartet exchange launches on qaux[1],
    // bra-shared exchange launches on qaux[2], range-walking exchange
    // launches on the batch stream
    hipStream_t qaux[3] = {nullptr, nullptr, nullptr};
    hipEvent_t qev[4] = {nullptr, nullptr, nullptr, nullptr};  // fork, join J, join small K, join bra-shared K
    std::vector<QGroup> qg;
    DevBuf<unsigned char> d_qtab;
    DevBuf<int4> d_qitems;
    std::vector<uint64_t> qgens;
    bool qplanned = false;
};

namespace {

constexpr int kBatchLanes = 8;
// Graph recording of batches.  Off: the recorded path ended in a host-side
// segmentation fault inside the batch call on the MI355X runtime, twice (the
// second time with no stream fork inside the recorded builds), and the cause
// is not yet shown; batches run the same fork/join with direct launches.
constexpr bool kBatchGraphs = false;

bool batch_ok(const eri_batch *b) { return b && b->magic == 0x4d4a4b42; }

void batch_release_graph(eri_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Record the batch into a graph (P/J/K pointers fixed in the nodes).
void batch_record(eri_batch *b)
{
    batch_release_graph(b);
    const size_t n = b->ctxs.size();
    for (eri_ctx *c : b->ctxs)
        if (c->opts.precision != ERI_FP64) ensure_mixed(c);  // allocations stay outside the capture
    HIPCHK(hipStreamSynchronize(b->st));
    for (eri_ctx *c : b->ctxs) {
        HIPCHK(hipStreamSynchronize(c->st));
        for (auto &x : c->aux) HIPCHK(hipStreamSynchronize(x));
    }
    std::vector<hipStream_t> saved(n);
    std::vector<bool> prof(n);
    HIPCHK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
    int rc = ERI_OK;
    try {
        HIPCHK(hipEventRecord(b->evs[0], b->st));
        for (size_t i = 0; i < n; ++i) {
            eri_ctx *c = b->ctxs[i];
            hipStream_t s = b->lanes[i % b->lanes.size()];
            HIPCHK(hipStreamWaitEvent(s, b->evs[0], 0));
            saved[i] = c->st;
            prof[i] = c->profile;
            c->st = s;
            c->profile = false;
            c->recording = true;  // molecules are the graph's parallel branches
            rc = build_jk(c, b->P[i], b->J[i], b->K[i]);
            c->recording = false;
            c->st = saved[i];
            c->profile = prof[i];
            if (rc) break;
        }
        if (!rc)
            for (size_t k = 0; k < b->lanes.size() && k < n; ++k) {
                HIPCHK(hipEventRecord(b->evs[1 + k], b->lanes[k]));
                HIPCHK(hipStreamWaitEvent(b->st, b->evs[1 + k], 0));
            }
    } catch (const HipError &e) {
        rc = e.code;
    }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->st, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        throw HipError{rc};
    }
    if (ec != hipSuccess) {
        set_err(ERI_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
        throw HipError{ERI_EHIP};
    }
    b->graph = g;
    HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    for (size_t i = 0; i < n; ++i) b->gens[i] = b->ctxs[i]->gen;
}

// Queue plan: every molecule's J-engine and exchange launches (as build_jk
// would issue them, in its precision mode: under ERI_MIXED* the double- and
// single-precision shares are separate launches of different kernels) are
// recorded instead of issued and
// grouped by kernel; each group becomes one launch whose items are the
// blocks of its molecules' launches, the launches with the most work per
// block first.  Rebuilt whenever a context changes.
void batch_plan_queue(eri_batch *b)
{
    b->qplanned = false;
    std::vector<eri_batch::QGroup> groups;
    std::vector<std::vector<std::pair<int, QueueRec>>> members;
    std::map<QueueLaunchFn, size_t> index;
    std::vector<QueueRec> recs;
    for (const int i : b->order) {
        eri_ctx *c = b->ctxs[(size_t)i];
        recs.clear();
        const bool mixed = c->opts.precision != ERI_FP64;
        if (mixed) {
            ensure_mixed(c);  // single-precision Hermite products, made on the context stream
            HIPCHK(hipStreamSynchronize(c->st));
        }
        const bool prof = c->profile;
        c->profile = false;
        queue_sink() = &recs;
        try {
            j_classes(c, mixed, nullptr);
            run_k(c, mixed, nullptr, nullptr, nullptr);
        } catch (...) {
            queue_sink() = nullptr;
            c->profile = prof;
            throw;
        }
        queue_sink() = nullptr;
        c->profile = prof;
        for (const QueueRec &r : recs) {
            if (!r.fn) {
                set_err(ERI_ESTATE, "no batch form of a %s launch (molecule %d)", r.kind, i);
                throw HipError{ERI_ESTATE};
            }
            auto it = index.find(r.fn);
            if (it == index.end()) {
                it = index.emplace(r.fn, groups.size()).first;
                groups.push_back(eri_batch::QGroup{r.fn, r.kind, 0, 0, 0, 0});
                members.emplace_back();
            }
            members[it->second].emplace_back(i, r);
        }
    }
    std::vector<unsigned char> tab;
    std::vector<int4> items;
    for (size_t g = 0; g < groups.size(); ++g) {
        auto &m = members[g];
        std::stable_sort(m.begin(), m.end(), [](const std::pair<int, QueueRec> &x, const std::pair<int, QueueRec> &y) {
            return x.second.work > y.second.work;
        });
        eri_batch::QGroup &q = groups[g];
        tab.resize((tab.size() + 255) / 256 * 256);
        q.tab_off = tab.size();
        q.item_off = items.size();
        int64_t count = 0;
        for (size_t e = 0; e < m.size(); ++e) {
            const QueueRec &r = m[e].second;
            tab.insert(tab.end(), r.args, r.args + r.asize);
            count += (int64_t)r.gx * r.gy;
            if (count > (int64_t)INT32_MAX) {
                set_err(ERI_EINVAL, "batch too large for one queue launch (%s: more than 2^31 blocks)", q.kind);
                throw HipError{ERI_EINVAL};
            }
            for (int by = 0; by < r.gy; ++by)
                for (int bx = 0; bx < r.gx; ++bx) items.push_back(make_int4((int)e, bx, by, r.gx));
        }
        q.nitems = (int)count;
        q.entries = (int)m.size();
    }
    b->d_qtab.alloc(0);
    b->d_qtab.upload(tab);
    b->d_qitems.upload(items);
    b->qg = std::move(groups);
    b->qgens.resize(b->ctxs.size());
    for (size_t i = 0; i < b->ctxs.size(); ++i) b->qgens[i] = b->ctxs[i]->gen;
    b->qplanned = true;
}

bool batch_queue_ready(const eri_batch *b)
{
    if (!b->qplanned) return false;
    for (size_t i = 0; i < b->ctxs.size(); ++i)
        if (b->qgens[i] != b->ctxs[i]->gen) return false;
    return true;
}

// One batch build with queue launches: every molecule's density transforms
// on the batch stream, the batch J-engine and exchange launches forked onto
// four streams as in build_jk and joined back, every molecule's output
// transforms on the batch stream.
void batch_build_queue(eri_batch *b, const double *const *P, double *const *J, double *const *K)
{
    if (!batch_queue_ready(b)) batch_plan_queue(b);
    const hipStream_t st = b->st;
    // under stream capture the timing events are left out (the build is then
    // a chain of kernel launches only)
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing(st, &cap));
    const bool timing = cap == hipStreamCaptureStatusNone;
    if (timing) HIPCHK(hipEventRecord(b->tev[0], st));
    for (const int i : b->order) {
        eri_ctx *c = b->ctxs[(size_t)i];
        const bool prof = c->profile;
        c->profile = false;
        const int nc = c->nbf_cart;
        const bool mixed = c->opts.precision != ERI_FP64;
        launch_p_to_cart(P[i], c->nbf, c->wk.Pc, nc, shell_map(c), c->opts.spherical, st);
        if (mixed || c->tau_dens > 0.0)
            launch_density_bounds(c->wk.Pc, nc, c->d_l.p, c->d_coff.p, c->nshell, c->d_Pm.p, c->d_cp.p, c->d_Q.p,
                                  (int)c->cp.size(), c->d_QD.p, st);
        c->built_mixed = mixed;
        c->mix_counts_ok = false;
        launch_fill_zero(c->wk.Jacc, (int64_t)nc * nc, st);
        launch_fill_zero(c->wk.Kacc, (int64_t)nc * nc, st);
        j_prologue(c, mixed, st);
        c->profile = prof;
    }
    HIPCHK(hipEventRecord(b->qev[0], st));
    HIPCHK(hipStreamWaitEvent(b->qaux[0], b->qev[0], 0));
    HIPCHK(hipStreamWaitEvent(b->qaux[1], b->qev[0], 0));
    HIPCHK(hipStreamWaitEvent(b->qaux[2], b->qev[0], 0));
    // at most 2^24 items per launch, so that items x lanes stays below the
    // 2^32 work-items of one launch
    constexpr int kMaxItems = 1 << 24;
    for (const eri_batch::QGroup &q : b->qg) {
        const bool jeng = std::strncmp(q.kind, "jeng", 4) == 0;
        const hipStream_t s = jeng ? b->qaux[0]
                              : std::strcmp(q.kind, "k_small") == 0 ? b->qaux[1]
                              : std::strcmp(q.kind, "k_pair") == 0  ? b->qaux[2]
                                                                    : st;
        for (int off = 0; off < q.nitems; off += kMaxItems)
            q.fn(b->d_qtab.p + q.tab_off, b->d_qitems.p + q.item_off + off, std::min(kMaxItems, q.nitems - off), s);
    }
    HIPCHK(hipEventRecord(b->qev[1], b->qaux[0]));
    HIPCHK(hipEventRecord(b->qev[2], b->qaux[1]));
    HIPCHK(hipEventRecord(b->qev[3], b->qaux[2]));
    HIPCHK(hipStreamWaitEvent(st, b->qev[1], 0));
    HIPCHK(hipStreamWaitEvent(st, b->qev[2], 0));
    HIPCHK(hipStreamWaitEvent(st, b->qev[3], 0));
    for (const int i : b->order) {
        eri_ctx *c = b->ctxs[(size_t)i];
        const bool prof = c->profile;
        c->profile = false;
        const int nc = c->nbf_cart;
        const ShellMap m = shell_map(c);
        j_epilogue(c, st);
        launch_acc_to_out(c->wk.Jacc, nc, J[i], c->nbf, m, c->opts.spherical, st);
        launch_acc_to_out(c->wk.Kacc, nc, K[i], c->nbf, m, c->opts.spherical, st);
        c->profile = prof;
        if (timing) HIPCHK(hipEventRecord(b->tev[1 + (size_t)i], st));
    }
    HIPCHK(hipGetLastError());
}

}  // namespace

namespace md {

std::vector<QueueRec> *&queue_sink()
{
    static thread_local std::vector<QueueRec> *sink = nullptr;
    return sink;
}

}  // namespace md

extern "C" {

int eri_batch_create(eri_ctx *const *ctxs, int32_t n, void *stream, eri_batch **out)
{
    g_err.clear();
    if (!out) return set_err(ERI_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctxs || n <= 0) return set_err(ERI_EINVAL, "no contexts (n=%d)", n);
    for (int i = 0; i < n; ++i)
        if (!ctx_ok(ctxs[i])) return set_err(ERI_ESTATE, "context %d invalid", i);
    for (int i = 1; i < n; ++i)
        if (ctxs[i]->device != ctxs[0]->device)
            return set_err(ERI_EINVAL, "context %d is on device %d, context 0 on device %d", i, ctxs[i]->device,
                           ctxs[0]->device);
    std::unique_ptr<eri_batch> b(new (std::nothrow) eri_batch);
    if (!b) return set_err(ERI_ENOMEM, "host allocation failed");
    try {
        b->ctxs.assign(ctxs, ctxs + n);
        b->gens.assign(n, ~0ull);
        // NULL is the default stream, as for eri_setup: the fork below records
        // its start event there and the join makes the default stream wait, so
        // work queued before and after the call on that stream stays ordered
        b->st = (hipStream_t)stream;
        b->lanes.resize(std::min(n, kBatchLanes));
        for (auto &s : b->lanes) HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        b->evs.resize(1 + b->lanes.size());
        for (auto &e : b->evs) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        b->tev.resize(1 + (size_t)n);
        for (auto &e : b->tev) HIPCHK(hipEventCreate(&e));
        for (auto &s : b->qaux) HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        for (auto &e : b->qev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        // largest molecules first, each onto the least-loaded lane (cost: the
        // spherical ERIs its unique quartets represent)
        b->order.resize(n);
        for (int i = 0; i < n; ++i) b->order[i] = i;
        std::stable_sort(b->order.begin(), b->order.end(),
                         [&](int x, int y) { return ctxs[x]->eris_sph > ctxs[y]->eris_sph; });
        b->lane_of.assign(n, 0);
        std::vector<double> load(b->lanes.size(), 0.0);
        for (int i : b->order) {
            const size_t k = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
            b->lane_of[i] = (int)k;
            load[k] += ctxs[i]->eris_sph;
        }
    } catch (const HipError &e) {
        return e.code;
    }
    *out = b.release();
    return ERI_OK;
}

int eri_batch_build_jk(eri_batch *b, const double *const *P, double *const *J, double *const *K)
{
    if (!batch_ok(b)) return set_err(ERI_ESTATE, "invalid batch");
    if (!P || !J || !K) return set_err(ERI_EINVAL, "null pointer array");
    const size_t n = b->ctxs.size();
    for (size_t i = 0; i < n; ++i) {
        if (!ctx_ok(b->ctxs[i])) return set_err(ERI_ESTATE, "context %zu destroyed", i);
        if (!P[i] || !J[i] || !K[i]) return set_err(ERI_EINVAL, "null P/J/K for molecule %zu", i);
    }
    try {
        if (b->mode == ERI_BATCH_QUEUE) {
            hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
            HIPCHK(hipStreamIsCapturing(b->st, &cap));
            if (cap != hipStreamCaptureStatusNone && !batch_queue_ready(b))
                return set_err(ERI_ESTATE, "batch queue plan must be made before stream capture (run one build "
                                           "outside the capture after each context change)");
            batch_build_queue(b, P, J, K);
            if (cap == hipStreamCaptureStatusNone) b->timed_once = true;
            return ERI_OK;
        }
        if (kBatchGraphs) {
            bool same = b->exec != nullptr && b->P.size() == n;
            for (size_t i = 0; same && i < n; ++i)
                if (b->P[i] != P[i] || b->J[i] != J[i] || b->K[i] != K[i] || b->gens[i] != b->ctxs[i]->gen)
                    same = false;
            if (!same) {
                b->P.assign(P, P + n);
                b->J.assign(J, J + n);
                b->K.assign(K, K + n);
                batch_record(b);
            }
            HIPCHK(hipGraphLaunch(b->exec, b->st));
        } else {
            // the same fork/join, launched directly: every molecule on one of
            // the batch's streams, all joined back into the batch stream
            HIPCHK(hipEventRecord(b->evs[0], b->st));
            HIPCHK(hipEventRecord(b->tev[0], b->st));
            for (auto &s : b->lanes) HIPCHK(hipStreamWaitEvent(s, b->evs[0], 0));
            for (const int i : b->order) {
                eri_ctx *c = b->ctxs[i];
                const hipStream_t saved = c->st;
                c->st = b->lanes[b->lane_of[i]];
                const int rc = build_jk(c, P[i], J[i], K[i]);
                c->st = saved;
                if (rc) return rc;
                HIPCHK(hipEventRecord(b->tev[1 + i], b->lanes[b->lane_of[i]]));
            }
            b->timed_once = true;
            for (size_t k = 0; k < b->lanes.size(); ++k) {
                HIPCHK(hipEventRecord(b->evs[1 + k], b->lanes[k]));
                HIPCHK(hipStreamWaitEvent(b->st, b->evs[1 + k], 0));
            }
        }
    } catch (const HipError &e) {
        return e.code;
    }
    return ERI_OK;
}

int eri_batch_set_mode(eri_batch *b, int32_t mode)
{
    if (!batch_ok(b)) return set_err(ERI_ESTATE, "invalid batch");
    if (mode != ERI_BATCH_QUEUE && mode != ERI_BATCH_STREAMS) return set_err(ERI_EINVAL, "unknown batch mode %d", mode);
    b->mode = mode;
    return ERI_OK;
}

int eri_batch_queue_info(eri_batch *b, int32_t *launches, int64_t *items)
{
    if (!batch_ok(b)) return set_err(ERI_ESTATE, "invalid batch");
    if (!launches || !items) return set_err(ERI_EINVAL, "null output");
    if (!b->qplanned) return set_err(ERI_ESTATE, "no queue build has run on this batch yet");
    *launches = (int32_t)b->qg.size();
    int64_t s = 0;
    for (const auto &q : b->qg) s += q.nitems;
    *items = s;
    return ERI_OK;
}

int eri_batch_latency(eri_batch *b, float *ms, int32_t n)
{
    if (!batch_ok(b)) return set_err(ERI_ESTATE, "invalid batch");
    if (!ms || n < 0) return set_err(ERI_EINVAL, "ms is NULL or n negative");
    if (!b->timed_once) return set_err(ERI_ESTATE, "no batch build has run with direct launches yet");
    try {
        for (int32_t i = 0; i < n && i < (int32_t)b->ctxs.size(); ++i) {
            HIPCHK(hipEventSynchronize(b->tev[1 + i]));
            HIPCHK(hipEventElapsedTime(&ms[i], b->tev[0], b->tev[1 + i]));
        }
    } catch (const HipError &e) {
        return e.code;
    }
    return ERI_OK;
}

int eri_batch_destroy(eri_batch *b)
{
    if (!b) return ERI_OK;
    if (!batch_ok(b)) return set_err(ERI_ESTATE, "invalid batch");
    (void)hipStreamSynchronize(b->st);
    batch_release_graph(b);
    for (auto &e : b->evs) (void)hipEventDestroy(e);
    for (auto &e : b->tev) (void)hipEventDestroy(e);
    for (auto &s : b->lanes) (void)hipStreamDestroy(s);
    for (auto &e : b->qev)
        if (e) (void)hipEventDestroy(e);
    for (auto &s : b->qaux)
        if (s) (void)hipStreamDestroy(s);
    b->magic = 0;
    delete b;
    return ERI_OK;
}

}  // extern "C"
