// queue.hpp -- batch launches: one launch per kernel for many molecules.
//
// A batch of contexts builds each angular class with ONE launch for all of
// its molecules: the blocks that every molecule's own launch of that kernel
// would have run become the items of the launch,
//     item = {entry, bx, by, gx}
// (entry indexes a table of the per-molecule argument structs; (bx, by) is
// the block of that molecule's launch and gx its grid width), ordered with
// the most work per block first.  Workgroup b runs item b, i.e. exactly the
// code of the block it stands for; the hardware dispatcher hands the items
// to compute units in order as they free up, so the long items start first
// and the short ones fill the tail.
//
// (A persistent form -- as many workgroups as the device holds, each pulling
// items from an atomic counter -- was tried first and dropped: in its item
// loop the compiler hoisted the body's constants out of the loop and spilled
// them in the larger classes, and the dispatcher already hands items out in
// order.)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "kern_args.hpp"

namespace md {

// A pointer loaded from the argument table is a generic (flat) pointer to
// the compiler, where the same field passed as a kernel argument is known to
// point to global memory; flat accesses are slower and, since they may reach
// LDS, make the compiler keep more values live (spills in the large classes).
// Rebuilding each pointer as a global one (an integer round trip into
// address space 1) gives the batch form the direct kernel's global loads and
// stores.
template <typename T>
__device__ __forceinline__ T *glob(T *p)
{
    auto g = (__attribute__((address_space(1))) T *)(uintptr_t)p;
    return (T *)g;
}

__device__ __forceinline__ void globalize(KArgs &a)
{
    a.bra = glob(a.bra); a.ket = glob(a.ket); a.rows = glob(a.rows); a.prefix = glob(a.prefix);
    a.pp = glob(a.pp); a.boys = glob(a.boys); a.D = glob(a.D); a.Kacc = glob(a.Kacc);
    a.eprod_bra = glob(a.eprod_bra); a.eprod_ket = glob(a.eprod_ket);
    a.eprodf_bra = glob(a.eprodf_bra); a.eprodf_ket = glob(a.eprodf_ket);
    a.Qbra = glob(a.Qbra); a.Qket = glob(a.Qket); a.Pm = glob(a.Pm);
}

__device__ __forceinline__ void globalize(KPArgs &a)
{
    a.bra = glob(a.bra); a.ket = glob(a.ket); a.chunks = glob(a.chunks); a.rows = glob(a.rows);
    a.prefix = glob(a.prefix); a.pp = glob(a.pp); a.boys = glob(a.boys); a.D = glob(a.D); a.Kacc = glob(a.Kacc);
    a.eprod_bra = glob(a.eprod_bra); a.eprod_ket = glob(a.eprod_ket);
    a.eprodf_bra = glob(a.eprodf_bra); a.eprodf_ket = glob(a.eprodf_ket);
    a.Qbra = glob(a.Qbra); a.Qket = glob(a.Qket); a.Pm = glob(a.Pm);
}

__device__ __forceinline__ void globalize(JArgs &a)
{
    a.pp = glob(a.pp); a.owner = glob(a.owner); a.Qbra = glob(a.Qbra); a.ket = glob(a.ket);
    a.Qket = glob(a.Qket); a.Dt = glob(a.Dt); a.Jh = glob(a.Jh); a.boys = glob(a.boys);
    a.Dtf = glob(a.Dtf); a.QDket = glob(a.QDket);
}

// Host side: a launch recorded instead of issued (see queue_sink); the
// function launches the batch form of the kernel over nitems items.
using QueueLaunchFn = void (*)(const void *tab, const int4 *items, int nitems, hipStream_t st);

struct QueueRec {
    QueueLaunchFn fn;      // launches the batch form of the kernel; groups launches
    int asize;             // bytes of one argument struct
    unsigned char args[512];
    int gx, gy;            // the grid the direct launch would have had
    double work;           // estimated work of one block, for the ordering
    const char *kind;      // kernel family, for names in statistics
};

// Non-null while a batch plan is recorded: the launchers of the J-engine and
// exchange kernels append their launch here instead of issuing it (double
// precision only: a single-precision launch is recorded with fn == nullptr,
// which the plan rejects).
std::vector<QueueRec> *&queue_sink();

template <typename A>
void queue_record(QueueLaunchFn fn, const A &a, int gx, int gy, double work, const char *kind)
{
    static_assert(sizeof(A) <= sizeof(QueueRec::args), "argument struct too large for a queue record");
    QueueRec r{};
    r.fn = fn;
    r.asize = (int)sizeof(A);
    __builtin_memcpy(r.args, &a, sizeof(A));
    r.gx = gx;
    r.gy = gy;
    r.work = work;
    r.kind = kind;
    queue_sink()->push_back(r);
}

// The launch function of batch kernel K with THREADS lanes per workgroup.
template <typename A, void (*K)(const A *__restrict__, const int4 *__restrict__), int THREADS>
void queue_launch(const void *tab, const int4 *items, int nitems, hipStream_t st)
{
    hipLaunchKernelGGL(K, dim3((unsigned)nitems), dim3(THREADS), 0, st, (const A *)tab, items);
}

}  // namespace md
