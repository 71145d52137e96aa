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
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/mdjk.h"
#include "launch.hpp"
#include "md_common.hpp"

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

// ---------------------------------------------------------------------------
// Boys table: F_m(i h) for m < kBoysNM.  For each grid point the top order
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
        tab.assign((size_t)kBoysNG * kBoysNM, 0.0);
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
                if (m < kBoysNM) tab[(size_t)i * kBoysNM + m] = (double)F;
            }
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

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    void alloc(size_t count)
    {
        release();
        n = count;
        if (count) HIPCHK(hipMalloc((void **)&p, count * sizeof(T)));
    }
    void upload(const std::vector<T> &h)
    {
        alloc(h.size());
        if (!h.empty()) HIPCHK(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    ~DevBuf() { release(); }
};

}  // namespace

struct eri_ctx {
    uint32_t magic = 0x4d444a4b;
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
    };
    std::vector<KWork> kwork;
    size_t dt_off[kPairClasses] = {}, jh_off[kPairClasses] = {};

    // device
    DevBuf<CPair> d_cp;
    DevBuf<double> d_Q;
    DevBuf<PrimPair> d_pp;
    DevBuf<int32_t> d_owner;
    DevBuf<int64_t> d_prefix;
    DevBuf<double> d_boys;
    DevBuf<double> d_Pc, d_Jacc, d_Kacc, d_Dt, d_Jh;
    DevBuf<int32_t> d_soc, d_sos, d_l, d_coff, d_soff;

    // stats
    int64_t n_quartets = 0;
    double eris_sph = 0, eris_cart = 0;
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
        if (o->precision != ERI_FP64 && o->precision != ERI_MIXED)
            return set_err(ERI_EINVAL, "unknown precision %d", o->precision);
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

    // 4. exchange work lists
    std::vector<int64_t> prefix;
    c->kwork.clear();
    c->n_quartets = 0;
    c->eris_sph = c->eris_cart = 0.0;
    for (int X = 0; X < kPairClasses; ++X)
        for (int Y = 0; Y <= X; ++Y) {
            eri_ctx::KWork w{X, Y, (int64_t)prefix.size(), 0};
            const double *QX = c->Q.data() + c->cp_base[X];
            const double *QY = c->Q.data() + c->cp_base[Y];
            const int nX = c->ncp[X], nY = c->ncp[Y];
            int64_t acc = 0;
            prefix.push_back(0);
            for (int i = 0; i < nX; ++i) {
                // kets with Q_i Q_j >= tau form a prefix of the descending list
                int lo = 0, hi = nY;
                while (lo < hi) {
                    int mid = (lo + hi) / 2;
                    if (QX[i] * QY[mid] >= tau) lo = mid + 1; else hi = mid;
                }
                int cnt = lo;
                if (X == Y) cnt = std::min(cnt, i + 1);
                acc += cnt;
                prefix.push_back(acc);
            }
            w.nwork = acc;
            c->kwork.push_back(w);
            c->n_quartets += acc;
            const int la = kPairL[X][0], lb = kPairL[X][1], lc = kPairL[Y][0], ld = kPairL[Y][1];
            c->eris_sph += (double)acc * nsph(la) * nsph(lb) * nsph(lc) * nsph(ld);
            c->eris_cart += (double)acc * ncart(la) * ncart(lb) * ncart(lc) * ncart(ld);
        }
    c->d_prefix.upload(prefix);

    // 5. Hermite density / Hermite J storage
    size_t dt = 0;
    for (int X = 0; X < kPairClasses; ++X) {
        c->dt_off[X] = dt;
        c->jh_off[X] = dt;
        dt += (size_t)c->npp[X] * nherm(kPairL[X][0] + kPairL[X][1]);
    }
    c->d_Dt.alloc(std::max<size_t>(dt, 1));
    c->d_Jh.alloc(std::max<size_t>(dt, 1));
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

void run_j(eri_ctx *c)
{
    hipStream_t st = c->st;
    const int nc = c->nbf_cart;
    for (int Y = 0; Y < kPairClasses; ++Y)
        launch_hermite_density(kPairL[Y][0], kPairL[Y][1], c->d_cp.p + c->cp_base[Y], c->ncp[Y], c->d_pp.p,
                               c->d_Pc.p, nc, c->d_Dt.p + c->dt_off[Y], c->pp_base[Y], st);
    launch_fill_zero(c->d_Jh.p, (int64_t)c->d_Jh.n, st);
    for (int X = 0; X < kPairClasses; ++X) {
        if (c->npp[X] == 0) continue;
        for (int Y = 0; Y < kPairClasses; ++Y) {
            if (c->ncp[Y] == 0) continue;
            JArgs a;
            a.pp = c->d_pp.p;
            a.owner = c->d_owner.p + c->pp_base[X];
            a.Qbra = c->d_Q.p + c->cp_base[X];
            a.pbase = c->pp_base[X];
            a.nbp = c->npp[X];
            a.ket = c->d_cp.p + c->cp_base[Y];
            a.Qket = c->d_Q.p + c->cp_base[Y];
            a.nket = c->ncp[Y];
            a.kchunk = 256;
            a.Dt = c->d_Dt.p + c->dt_off[Y];
            a.dt_base = c->pp_base[Y];
            a.Jh = c->d_Jh.p + c->jh_off[X];
            a.boys = c->d_boys.p;
            a.tau = c->opts.schwarz_thresh;
            a.tau_prim = c->opts.prim_thresh;
            launch_jeng(kPairL[X][0] + kPairL[X][1], kPairL[Y][0] + kPairL[Y][1], a, st);
        }
    }
    for (int X = 0; X < kPairClasses; ++X)
        launch_hermite_to_cart(kPairL[X][0], kPairL[X][1], c->d_cp.p + c->cp_base[X], c->ncp[X], c->d_pp.p,
                               c->d_Jh.p + c->jh_off[X], c->pp_base[X], c->d_Jacc.p, nc, st);
}

void run_k(eri_ctx *c)
{
    hipStream_t st = c->st;
    for (const auto &w : c->kwork) {
        if (w.nwork == 0) continue;
        KArgs a;
        a.bra = c->d_cp.p + c->cp_base[w.X];
        a.ket = c->d_cp.p + c->cp_base[w.Y];
        a.prefix = c->d_prefix.p + w.off;
        a.nwork = w.nwork;
        a.nbra = c->ncp[w.X];
        a.same = w.X == w.Y;
        a.pp = c->d_pp.p;
        a.boys = c->d_boys.p;
        a.D = c->d_Pc.p;
        a.Kacc = c->d_Kacc.p;
        a.ld = c->nbf_cart;
        a.tau_prim = c->opts.prim_thresh;
        const int la = kPairL[w.X][0], lb = kPairL[w.X][1], lc = kPairL[w.Y][0], ld = kPairL[w.Y][1];
        bool ok = launch_k_small(la, lb, lc, ld, a, st) || launch_k_wave_0(la, lb, lc, ld, a, st) ||
                  launch_k_wave_1(la, lb, lc, ld, a, st) || launch_k_wave_2(la, lb, lc, ld, a, st) ||
                  launch_k_wave_3(la, lb, lc, ld, a, st) || launch_k_wave_4(la, lb, lc, ld, a, st) ||
                  launch_k_wave_5(la, lb, lc, ld, a, st);
        if (!ok) {
            set_err(ERI_ESTATE, "no exchange kernel for class (%d%d|%d%d)", la, lb, lc, ld);
            throw HipError{ERI_ESTATE};
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
    if (precision != ERI_FP64 && precision != ERI_MIXED) return set_err(ERI_EINVAL, "unknown precision %d", precision);
    if (!(mixed_thresh >= 0.0)) return set_err(ERI_EINVAL, "negative mixed threshold");
    ctx->opts.precision = precision;
    ctx->opts.mixed_thresh = mixed_thresh;
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
        launch_p_to_cart(P, ctx->nbf, ctx->d_Pc.p, nc, m, ctx->opts.spherical, st);
        if (J) {
            launch_fill_zero(ctx->d_Jacc.p, (int64_t)nc * nc, st);
            run_j(ctx);
            launch_acc_to_out(ctx->d_Jacc.p, nc, J, ctx->nbf, m, ctx->opts.spherical, st);
        }
        if (K) {
            launch_fill_zero(ctx->d_Kacc.p, (int64_t)nc * nc, st);
            run_k(ctx);
            launch_acc_to_out(ctx->d_Kacc.p, nc, K, ctx->nbf, m, ctx->opts.spherical, st);
        }
        HIPCHK(hipGetLastError());
    } catch (const HipError &e) {
        return e.code;
    }
    return ERI_OK;
}

int jk_grad(eri_ctx *ctx, const double *P, double *grad, double *E)
{
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    (void)P; (void)grad; (void)E;
    return set_err(ERI_ESTATE, "jk_grad is not available in this build");
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
    out->eris_sph = ctx->eris_sph;
    out->eris_cart = ctx->eris_cart;
    out->last_ms = ctx->last_ms;
    return ERI_OK;
}

int eri_destroy(eri_ctx *ctx)
{
    if (!ctx) return ERI_OK;
    if (!ctx_ok(ctx)) return set_err(ERI_ESTATE, "invalid context");
    if (ctx->st) (void)hipStreamSynchronize(ctx->st); else (void)hipDeviceSynchronize();
    ctx->magic = 0;
    delete ctx;
    return ERI_OK;
}

const char *eri_last_error(void) { return g_err.c_str(); }

}  // extern "C"
