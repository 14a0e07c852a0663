// Internal data structures shared by the host side and the gfx950 kernels of
// libislf.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/islf.h"

namespace islf {

constexpr int kBlock = 256;          // threads per workgroup of the update kernels
constexpr int kAccSlots = 64;        // spread of the per-sweep partial-sum atomics
constexpr int kClasses = 4;          // bulk, x = 0, x = Lx-1, one-layer film
constexpr int kThrPerClass = 16;     // index u*8 + cnt, cnt in 0..6
constexpr int kThrEntries = kClasses * kThrPerClass;
constexpr int kPadEntry = kThrEntries - 1;   // class 3, u = 1, cnt = 7: never a real site
constexpr int kMaxMarch = 256;       // x planes one thread may march through per entry
constexpr int kNoAllocMaxReps = 8192;   // live replicas islf_means_noalloc serves per call

// One item of work for one replica.  j counts 8-byte columns of one
// sublattice row (int8 format: 8 sites) or 32-bit words of one sublattice
// row (bit-packed: 32 sites).
// Main tile (kind 0, rows 2 .. Ly-2): a box of rows/columns starting at
// (x0, y0, j0) whose extent is the replica's tile shape, or (linear tile
// shape, i8_tj = 0) the columns [y0, j0) of a plane's main rows in row-major
// order, marched through nsteps x planes from x0 (a launch plan may cut a
// tile into pieces along x).
// Seam-slab tile (kind 1, rows Ly-1, 0, 1): x0 = first x pair p (planes p and
// Lx-1-p), y0 = number of consecutive pairs, j0 = first column,
// nsteps = number of columns.
enum { ITEM_MAIN = 0, ITEM_SLAB = 1 };
struct Entry {
    int32_t rep, x0, y0, j0;
    int32_t nsteps, kind;
};

// Launch kinds of a run of sweeps and their flags.
enum { KIND_A = 0, KIND_B = 1, KIND_F = 2 };
enum { FLAG_PREV = 1, FLAG_FOLD = 2 };   // A: do the previous sweep's phase 3; B: fold its record

// Read-only description of a replica as the kernels see it.
struct RepDesc {
    uint8_t *spins;        // int8 format: byte 1 = up, 0 = down; rows of RB = 2*Hp bytes (even z, odd z)
                           // bit-packed: rows of 2*Wq uint32 words (even z, odd z)
    islf_obs *rec;         // ring of cap per-sweep records
    long long *acc;        // 2 x kAccSlots x 4 partial sums (double-buffered by t & 1)
    uint64_t thr[kThrEntries];  // acceptance thresholds, index class*16 + u*8 + cnt
    uint32_t thr_m1[kThrEntries];  // thr - 1 (accept iff u <= thr_m1) where thr >= 1
    int32_t dpack[kThrEntries];    // change of (B, M) on a flip: dB + 65536 * dM
    uint64_t never_mask;           // bit i set when thr[i] == 0 (no draw can accept)
    int32_t Lx, Ly, Lz;
    int32_t C;             // Philox groups of 8 consecutive z per row, ceil(Lz/8)
    int32_t K;             // int8 8-byte columns per sublattice row, ceil(Lz/16)
    int32_t Hp;            // int8 bytes per sublattice row, 8*K
    int32_t RB;            // int8 row stride in bytes, 2*Hp
    int32_t Wq;            // bit-packed words per sublattice row, ceil(Lz/64)
    int32_t seam_reflect;  // 1: the y seam maps x -> Lx-1-x
    int32_t seam_invert;   // 1: the y seam carries eps = -1
    uint32_t key0, key1, replica, cap;
    int32_t fmt;                   // islf_spin_format
    int32_t i8_tj, i8_ty, i8_mx;   // main tiles: columns x rows per workgroup (0 x 0: linear), x planes marched
    double J, H, h1, hn;           // for energies (Eq. 1)
};

// Mutable per-replica state (device memory).
struct RepState {
    long long cur[4];      // observables after the last completed sweep
    uint32_t t;            // completed sweeps
    uint32_t live;
    uint32_t pad_[2];
};

// Persistent-kernel synchronisation words (device memory, zero-initialised).
// Two-level grid barrier state.  Blocks arrive at their group's counter; the
// last arrival of a group arrives at the top counter, waits for all groups,
// then bumps its group's release counter, which the group's other blocks
// poll.  Every counter only changes through read-modify-write atomics and is
// re-zeroed by a fill kernel before each persistent launch; each sits on its
// own 128-byte line.
// 256 blocks per group (3 to 5 groups at the usual grids) measured best:
// 2-5% over 32, 64 or one flat group of 1024
constexpr int kBarrierGroup = 256;    // blocks per group
constexpr int kMaxGroups = 16;        // up to 4096 blocks
struct SyncLine {
    unsigned long long v;
    unsigned long long pad_[15];
};
struct GridSync {
    SyncLine top;
    SyncLine error;
    SyncLine arrive[kMaxGroups];
    SyncLine release[kMaxGroups];
};

// Team form of the persistent kernel: every workgroup serves one replica
// (its team), and a team's workgroups meet at a barrier of their own (an
// arrival and a release counter per replica slot, each on its own line,
// re-zeroed before each launch), so replicas do not wait for each other.
struct TeamInfo {
    int32_t rep;    // replica slot
    int32_t rank;   // 0 .. size-1 inside the team (rank 0 folds the records)
    int32_t size;   // workgroups of the team
    int32_t pad_;
};

}  // namespace islf
