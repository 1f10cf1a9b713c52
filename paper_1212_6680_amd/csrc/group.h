// Grouped launches: one launch runs the same kernel body for several
// independent problems (boxes), each with its own arguments and grid.
//
// Every kernel that can be grouped is written as a __device__ body taking its
// argument block and a Blk (the block's coordinates and grid size).  The
// plain kernel passes the hardware blockIdx/gridDim; the grouped kernel
// (suffix _grp) takes a table of GroupEntry records, finds the entry owning
// its flat block index (entries are sorted by their first block), and runs
// the body with that entry's arguments and local block coordinates.  An entry
// may name a device flag; when the flag is zero the entry's blocks return at
// once (a converged Krylov solve stops doing work without changing the
// launch sequence, so the sequence can be captured in a HIP graph).
//
// Host side: while a recorder is installed (g_rec), launch sites append
// (grouped kernel, grid, block, LDS bytes, argument bytes) instead of
// launching.
#pragma once

#include <array>
#include <cstring>
#include <vector>

#include "smg_internal.h"

namespace smg {

struct Blk {
    int x, y, z;
    int gx, gy, gz;
};

#define SMG_BLK_HW                                                                                             \
    smg::Blk                                                                                                   \
    {                                                                                                          \
        static_cast<int>(blockIdx.x), static_cast<int>(blockIdx.y), static_cast<int>(blockIdx.z),              \
            static_cast<int>(gridDim.x), static_cast<int>(gridDim.y), static_cast<int>(gridDim.z)              \
    }

// The workgroups of a launch are dealt to the 8 XCDs round-robin by flat id,
// and each XCD has its own L2.  This renumbering gives every XCD one
// contiguous range of the logical order (x fastest), so neighbouring tiles
// that read each other's halo lines, or the planes next to theirs, run under
// the same L2.  It is a bijection of the flat ids for any grid size.
__device__ inline Blk blk_xcd()
{
    constexpr int kXcd = 8;
    const int gx = static_cast<int>(gridDim.x), gy = static_cast<int>(gridDim.y), gz = static_cast<int>(gridDim.z);
    const int nb = gx * gy * gz;
    const int l = static_cast<int>(blockIdx.x) + gx * (static_cast<int>(blockIdx.y) + gy * static_cast<int>(blockIdx.z));
    const int q = nb / kXcd, rem = nb % kXcd, x = l % kXcd;
    const int lp = x * q + min(x, rem) + l / kXcd;
    return Blk{lp % gx, (lp / gx) % gy, lp / (gx * gy), gx, gy, gz};
}

#define SMG_BLK_XCD smg::blk_xcd()

constexpr int kGroupArgBytes = 528;

struct alignas(16) GroupEntry {
    int start;              // first flat block of this entry
    int gx, gy, gz;         // the entry's own grid
    const int *active;      // nullable: skip when *active == 0
    long long pad;
    unsigned char args[kGroupArgBytes];
};

template <class Args>
__device__ inline bool group_entry(const GroupEntry *tab, int n, const Args *&a, Blk &blk)
{
    const int b = static_cast<int>(blockIdx.x);
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].start <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    const GroupEntry &e = tab[lo];
    if (e.active && *e.active == 0) return false;
    const int l = b - e.start;
    blk = Blk{l % e.gx, (l / e.gx) % e.gy, l / (e.gx * e.gy), e.gx, e.gy, e.gz};
    a = reinterpret_cast<const Args *>(e.args);
    return true;
}

// A recorded launch.
struct LaunchRec {
    const void *kg;         // grouped kernel
    dim3 grid, block;
    unsigned lds;
    const int *active;
    std::array<unsigned char, kGroupArgBytes> args;
};

template <class Args>
inline void record_launch(const void *kg, dim3 grid, dim3 block, size_t lds, const Args &a)
{
    static_assert(sizeof(Args) <= kGroupArgBytes, "argument block too large for a group entry");
    LaunchRec r{};
    r.kg = kg;
    r.grid = grid;
    r.block = block;
    r.lds = static_cast<unsigned>(lds);
    r.active = nullptr;
    std::memcpy(r.args.data(), &a, sizeof(Args));
    g_rec->push_back(r);
}

}  // namespace smg

// Launch K with ARGS, or record its grouped twin KG while a recorder is installed.
#define SMG_LAUNCH_G(EV, K, KG, G, B, L, S, ARGS)                                                             \
    do {                                                                                                       \
        if (smg::g_rec)                                                                                        \
            smg::record_launch(reinterpret_cast<const void *>(KG), G, B, L, ARGS);                            \
        else                                                                                                   \
            SMG_LAUNCH(EV, K, G, B, L, S, ARGS);                                                               \
    } while (0)
