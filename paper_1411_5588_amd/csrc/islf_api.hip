// Host side of libislf: the C ABI declared in include/islf.h.
//
// Owns contexts (replica slots, device buffers, work lists), builds the
// Metropolis threshold tables in IEEE double (Sec. II.A Eq. 1 energy change,
// acceptance min(1, exp(-beta dE)) on a uint32 draw), and issues the kernels
// of islf_kernels.hip in the plain, batched or persistent form, optionally as
// a captured HIP graph.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <unordered_map>
#include <vector>

#include "islf_internal.h"

namespace islf {
hipError_t launch_sweep(int fmt, int kind, const RepDesc *descs, RepState *st, const Entry *items,
                        const int *first, int grid, const int *reps, int n_reps, uint32_t s, uint32_t flags,
                        hipStream_t strm);
hipError_t sweep_blocks_per_cu(int fmt, int *per_cu);
hipError_t launch_fold(const RepDesc *descs, RepState *st, const int *reps, int n_reps, uint32_t s,
                       uint32_t advance, hipStream_t strm);
const void *persistent_kernel(int fmt);
const void *persistent_teams_kernel(int fmt);
hipError_t launch_persistent(int fmt, const RepDesc *descs, RepState *st, const Entry *items, const int *first,
                             const int *reps, int nreps, uint32_t nsweeps, GridSync *sync, int grid, hipStream_t s);
hipError_t launch_persistent_teams(int fmt, const RepDesc *descs, RepState *st, const Entry *items, const int *first,
                                   const TeamInfo *teams, uint32_t nsweeps, GridSync *sync, SyncLine *rsync,
                                   int n_rsync, int grid, hipStream_t s);
hipError_t launch_init(int fmt, const RepDesc *descs, int rep, int mode, const int8_t *host, hipStream_t s);
hipError_t launch_export(const RepDesc *descs, int rep, long rows, int8_t *out, hipStream_t s);
hipError_t launch_recompute(const RepDesc *descs, int rep, long rows, const int8_t *spins, unsigned long long *out,
                            hipStream_t s);
hipError_t launch_set_state(RepState *st, int rep, const unsigned long long *obs, uint32_t t, hipStream_t s);
hipError_t launch_layer_profile(const RepDesc *descs, int rep, long rows, long words_per_row, int32_t *out,
                                long long *acc, hipStream_t s);
hipError_t launch_zero(unsigned long long *p, long n, hipStream_t s);
hipError_t launch_energy(const islf_obs *rec, uint32_t cap, uint64_t first, uint32_t count, double J,
                         double H, double h1, double hn, double *out, hipStream_t s);
hipError_t launch_means(const RepDesc *descs, const int *reps, int n, uint64_t first, uint32_t count,
                        double *out, hipStream_t s);
hipError_t launch_integrate(const double *h, const double *m1, const double *mn, int n, double c1, double cn,
                            double norm, double *out, hipStream_t s);
hipError_t noalloc_scratch(double **out);
}  // namespace islf

using namespace islf;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static islf_status fail(islf_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(ISLF_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

extern "C" const char *islf_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// tile variants (main tiles, rows 2 .. Ly-2, both formats): a workgroup owns
// tj columns x ty rows (tj*ty <= 256 threads) and each thread marches through
// mx x planes; a column is an 8-byte column of a sublattice half-row (int8)
// or a 32-bit word of a sublattice row (bit-packed), and tj is the most even split of a row's
// columns into pieces of at most tj_max.  Seam-slab tiles (rows Ly-1, 0, 1):
// np mirror pairs of x planes x nj columns with np*nj <= 128, so that a row
// stage has at most one task per thread.
// ---------------------------------------------------------------------------
struct I8Tile {
    int tj_max, mx;
};
// tj_max = 0: linear tiles (a workgroup takes kBlock consecutive columns of
// a plane's main rows in row-major order, whatever the row length)
static const I8Tile kI8Tiles[] = {
    {16, 16}, {32, 16}, {64, 16}, {128, 16}, {256, 16}, {16, 8},  {32, 8},   {64, 8},
    {16, 32}, {32, 32}, {64, 32}, {128, 32}, {16, 64}, {32, 64}, {64, 64}, {256, 64},
    {0, 16},  {0, 8},   {0, 32},  {0, kMaxMarch},
};
static const I8Tile kBpTilesM[] = {
    {16, 4}, {32, 4}, {64, 4}, {8, 4}, {4, 4}, {16, 2}, {16, 8}, {32, 8}, {8, 8}, {64, 8}, {4, 8}, {16, 16},
    {0, 4},  {0, 2},  {0, 8},  {0, kMaxMarch},
};
static const int kNumBpTilesM = (int)(sizeof(kBpTilesM) / sizeof(kBpTilesM[0]));
static const int kNumI8Tiles = (int)(sizeof(kI8Tiles) / sizeof(kI8Tiles[0]));

static int num_tiles_of(int fmt) { return fmt == ISLF_SPIN_INT8 ? kNumI8Tiles : kNumBpTilesM; }

static long ceil_div(long a, long b) { return (a + b - 1) / b; }

// Columns of one sublattice row a thread takes: 8-byte columns (8 sites,
// int8) or 32-bit words (32 sites, bit-packed).
static long columns_of(const islf_replica_desc &d, int fmt)
{
    return fmt == ISLF_SPIN_INT8 ? (d.Lz + 15) / 16 : (d.Lz + 63) / 64;
}

struct I8Shape {
    int tj, ty, mx;
};
static I8Shape i8_shape(const islf_replica_desc &d, int tile, int fmt = ISLF_SPIN_INT8)
{
    const long C = columns_of(d, fmt);
    const I8Tile &t = fmt == ISLF_SPIN_INT8 ? kI8Tiles[tile] : kBpTilesM[tile];
    I8Shape s;
    s.mx = std::min(t.mx, d.Lx);
    if (t.tj_max == 0) {
        s.tj = s.ty = 0;
        return s;
    }
    const long pieces = ceil_div(C, t.tj_max);
    s.tj = (int)ceil_div(C, pieces);
    s.ty = (int)std::min<long>(kBlock / s.tj, std::max(1, d.Ly - 3));
    return s;
}

// fraction of a plane's thread slots that own a real column / word (the x
// extent costs nothing: plans cut tiles by x steps)
static double tile_efficiency(const islf_replica_desc &d, int fmt, int tile)
{
    const double ny = d.Ly - 3;
    if (ny <= 0) return 1.0;
    const long C = columns_of(d, fmt);
    const I8Shape s = i8_shape(d, tile, fmt);
    const double per_plane = s.tj == 0 ? (double)ceil_div((long)ny * C, kBlock)
                                       : (double)ceil_div((long)ny, s.ty) * ceil_div(C, s.tj);
    return ny * C / (per_plane * kBlock);
}

// The variant with the fewest idle thread slots among the default x extents
// (16 planes int8, 4 bit-packed) and the linear tile over the whole x range;
// that one wins ties: a workgroup's share of a plan is then mostly one
// contiguous piece, with one set-up (view, tables, first loads, flush)
// instead of one per tile.
static int default_tile(const islf_replica_desc *d, int fmt)
{
    double best = -1.0;
    int best_i = 0;
    for (int i = 0; i < num_tiles_of(fmt); ++i) {
        const I8Tile &t = fmt == ISLF_SPIN_INT8 ? kI8Tiles[i] : kBpTilesM[i];
        const bool whole = t.tj_max == 0 && t.mx == kMaxMarch;
        if (!whole && t.mx != (fmt == ISLF_SPIN_INT8 ? 16 : 4)) continue;
        const double eff = tile_efficiency(*d, fmt, i);
        if (eff > best + 1e-9 || (whole && eff > best - 1e-9)) {
            best = std::max(best, eff);
            best_i = i;
        }
    }
    return best_i;
}

struct SlabShape {
    int np, nj;
};
// the (pairs, columns) split with the fewest idle thread slots, then the
// fewest entries
static SlabShape slab_shape(const islf_replica_desc &d, int fmt)
{
    const long J = columns_of(d, fmt);
    const long P = (d.Lx + 1) / 2;
    const long cap = kBlock / 2;
    SlabShape best{1, 1};
    long best_cost = -1;
    for (long pieces = ceil_div(J, cap); pieces <= J; ++pieces) {
        const long nj = ceil_div(J, pieces);
        if (ceil_div(J, nj) != pieces) continue;
        const long np0 = std::min(P, std::max(1l, cap / nj));
        const long np = ceil_div(P, ceil_div(P, np0));
        const long entries = ceil_div(P, np) * pieces;
        const long cost = entries * cap;   // thread slots of one row stage
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = SlabShape{(int)np, (int)nj};
        }
    }
    return best;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct Replica {
    islf_replica_desc desc{};
    bool live = false;
    void *mem = nullptr;     // spins | records | accumulators
    size_t mem_bytes = 0;
    uint64_t t_host = 0;     // sweeps issued so far
    bool failed = false;     // its chain was cut short by a failed persistent launch
    int tile = 0;
    RepDesc d{};
    std::vector<Entry> main, slab;
};

// A launch plan: `grid` workgroups, workgroup b running items
// [first[b], first[b+1]) (device arrays); slab items come first and sit in
// workgroups [0, slab_grid).
struct Plan {
    Entry *items = nullptr;
    int *first = nullptr;
    long items_cap = 0, first_cap = 0;
    int grid = 0, slab_grid = 0;
    bool valid = false;
};

struct islf_ctx {
    int fmt = 0;
    uint32_t cap = 0;
    hipStream_t stream = nullptr;
    islf_alloc_fn alloc = nullptr;
    islf_free_fn free_fn = nullptr;
    void *user = nullptr;
    int exec = ISLF_EXEC_BATCHED;
    int num_cu = 0;
    int resident_slots = 0;    // workgroups of the sweep kernels resident at once on the device
    int sweep_slots = 0;       // default workgroups per sweep launch (2 per resident slot)
    int grid_override = 0;     // workgroups per batched / plain launch (0: sweep_slots)
    double taper_override = -1.0;   // share taper of the batched and persistent plans (< 0: the built-in one)
    int persistent_grid = 0;   // workgroups of the persistent kernel's cooperative launch
    int persistent_bound = 0;  // co-residency bound computed for it on this device
    double *noalloc_scratch = nullptr;   // this device's copy of the means scratch array

    std::vector<Replica> reps;
    int slot_capacity = 0;
    RepDesc *d_desc = nullptr;
    RepState *d_state = nullptr;
    GridSync *d_sync = nullptr;
    // team form of the persistent plan: per-workgroup team records and one
    // arrival counter per replica slot
    bool persistent_teams = false;
    TeamInfo *d_teams = nullptr;
    long teams_cap = 0;
    SyncLine *d_rsync = nullptr;
    int rsync_cap = 0;
    int team_mode = -1;        // 1: team barriers when every live replica can have a workgroup; 0: grid; -1: automatic
    unsigned long long *d_scratch = nullptr;   // 64 x u64
    int *d_live = nullptr;                      // live replica ids
    int live_capacity = 0;
    Plan batched, persistent;
    std::vector<Plan> plain;                    // per slot
    // batched form with concurrent replica groups: group g sweeps its
    // replicas on side_stream[g], a stream the context creates; the
    // context's stream only forks them and joins them
    int groups_req = 0;                         // 0: automatic
    bool groups_valid = false;
    std::vector<Plan> group_plan;
    std::vector<int> group_off, group_len;      // into d_group_live
    int *d_group_live = nullptr;
    int group_live_cap = 0;
    std::vector<hipStream_t> side_stream;       // group g issues on side_stream[g]
    std::vector<hipEvent_t> side_event;         // [0] fork, [g+1] join of group g
    std::vector<int> live;
    bool dirty = true;

    // captured sweeps: one single-stream graph per concurrent group (one
    // graph otherwise), replayed on the group's stream
    std::vector<hipGraph_t> graphs;
    std::vector<hipGraphExec_t> graph_execs;
    uint32_t graph_sweeps = 0;
    bool graph_valid = false;

    // device bytes the context holds, by allocation
    std::unordered_map<void *, size_t> alloc_bytes;
    size_t dev_bytes = 0;
};

static islf_status check_intact(islf_ctx *c, int rep);
static islf_status check_none_failed(const islf_ctx *c);

static void *dev_alloc(islf_ctx *c, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (c->alloc) p = c->alloc(bytes, c->user);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (p) {
        c->alloc_bytes[p] = bytes;
        c->dev_bytes += bytes;
    }
    return p;
}

static void dev_free(islf_ctx *c, void *p)
{
    if (!p) return;
    auto it = c->alloc_bytes.find(p);
    if (it != c->alloc_bytes.end()) {
        c->dev_bytes -= it->second;
        c->alloc_bytes.erase(it);
    }
    if (c->free_fn) c->free_fn(p, c->user);
    else (void)hipFree(p);
}

// ---------------------------------------------------------------------------
// validation, sizes, thresholds
// ---------------------------------------------------------------------------
static islf_status validate(const islf_replica_desc *d)
{
    if (!d) return fail(ISLF_EINVAL, "NULL replica descriptor");
    if (d->Lx < 1 || d->Ly < 2 || d->Lz < 2 || (d->Lz & 1))
        return fail(ISLF_EINVAL, "invalid shape %dx%dx%d (need Lx>=1, Ly>=2, Lz>=2 even)", d->Lx, d->Ly, d->Lz);
    if (d->ybc < 0 || d->ybc > 2) return fail(ISLF_EINVAL, "invalid y boundary %d", d->ybc);
    if (d->init < 0 || d->init > 3) return fail(ISLF_EINVAL, "invalid init mode %d", d->init);
    if (!(d->beta >= 0.0)) return fail(ISLF_EINVAL, "beta must be >= 0 (got %g)", d->beta);
    if (!isfinite(d->J) || !isfinite(d->H) || !isfinite(d->h1) || !isfinite(d->hn))
        return fail(ISLF_EINVAL, "J, H, h1, hn must be finite");
    const unsigned long long rows = (unsigned long long)d->Lx * (unsigned long long)d->Ly;
    const unsigned long long groups = rows * (unsigned long long)((d->Lz + 7) / 8);   // Philox groups of 8 z
    if (groups * 2ull > (1ull << 32))
        return fail(ISLF_ERANGE, "lattice %dx%dx%d exceeds the 32-bit Philox group counter", d->Lx, d->Ly, d->Lz);
    if (rows * 16ull * (unsigned long long)((d->Lz + 15) / 16) >= (1ull << 32))
        return fail(ISLF_ERANGE, "lattice %dx%dx%d exceeds 4 GiB of int8 spins", d->Lx, d->Ly, d->Lz);
    return ISLF_OK;
}

static size_t spin_bytes(const islf_replica_desc *d, int fmt)
{
    const size_t rows = (size_t)d->Lx * d->Ly;
    if (fmt == ISLF_SPIN_INT8) return rows * 16 * (size_t)((d->Lz + 15) / 16);
    return rows * 2 * 4 * (size_t)((d->Lz + 63) / 64);
}

static size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static size_t replica_bytes(const islf_replica_desc *d, int fmt, uint32_t cap)
{
    return round_up(spin_bytes(d, fmt), 256) + round_up((size_t)cap * sizeof(islf_obs), 256) +
           2 * kAccSlots * 4 * sizeof(long long);
}

// thr = 2^32 if dE <= 0 else floor(2^32 exp(-beta dE)), with
// dE = 2 s (J n + h), n = 2*cnt - k, h the field of the site's layer.
// Alongside: thr - 1 as 32 bits, the packed change (dB, dM) = (-2 s n, -2 s)
// of a flip as dB + 65536 dM, and the set of moves that can never be taken.
static void build_tables(const islf_replica_desc *d, RepDesc &D)
{
    uint64_t *thr = D.thr;
    D.never_mask = 0;
    for (int c = 0; c < kClasses; ++c) {
        double h = d->H;
        if (c & 1) h = h + d->h1;
        if (c & 2) h = h + d->hn;
        const int k = 6 - ((c & 1) ? 1 : 0) - ((c & 2) ? 1 : 0);
        for (int u = 0; u < 2; ++u) {
            const int s = 2 * u - 1;
            for (int cnt = 0; cnt < 8; ++cnt) {
                uint64_t v = 0;
                int32_t dp = 0;
                const int i = c * kThrPerClass + u * 8 + cnt;
                if (cnt <= k) {
                    const int n = 2 * cnt - k;
                    const double dE = 2.0 * (double)s * (d->J * (double)n + h);
                    if (dE <= 0.0) v = 1ull << 32;
                    else v = (uint64_t)floor(ldexp(exp(-(d->beta * dE)), 32));
                    dp = (-2 * s * n) + 65536 * (-2 * s);
                    if (v == 0) D.never_mask |= 1ull << i;
                }
                thr[i] = v;
                D.thr_m1[i] = v ? (uint32_t)(v - 1) : 0u;
                D.dpack[i] = dp;
            }
        }
    }
}

static void build_work(Replica &R, int rep_id, int fmt)
{
    const islf_replica_desc &d = R.desc;
    R.main.clear();
    R.slab.clear();
    const int J = (int)columns_of(d, fmt);
    const I8Shape s = i8_shape(d, R.tile, fmt);
    const int cols = std::max(0, d.Ly - 3) * J;   // main columns of a plane (rows 2 .. Ly-2)
    for (int x0 = 0; x0 < d.Lx; x0 += s.mx) {
        if (s.tj == 0) {
            // linear tile: y0 = first column, j0 = end of the range
            for (int c0 = 0; c0 < cols; c0 += kBlock)
                R.main.push_back(Entry{rep_id, x0, c0, std::min(c0 + kBlock, cols), std::min(s.mx, d.Lx - x0),
                                       ITEM_MAIN});
            continue;
        }
        for (int y0 = 2; y0 < d.Ly - 1; y0 += s.ty)
            for (int j0 = 0; j0 < J; j0 += s.tj)
                R.main.push_back(Entry{rep_id, x0, y0, j0, std::min(s.mx, d.Lx - x0), ITEM_MAIN});
    }
    R.d.i8_tj = s.tj;
    R.d.i8_ty = s.ty;
    R.d.i8_mx = s.mx;
    const SlabShape sl = slab_shape(d, fmt);
    const int P = (d.Lx + 1) / 2;
    for (int p0 = 0; p0 < P; p0 += sl.np)
        for (int j0 = 0; j0 < J; j0 += sl.nj)
            R.slab.push_back(Entry{rep_id, p0, std::min(sl.np, P - p0), j0, std::min(sl.nj, J - j0), ITEM_SLAB});
}

static void fill_desc(Replica &R, int fmt, uint32_t cap)
{
    const islf_replica_desc &d = R.desc;
    RepDesc &D = R.d;
    uint8_t *m = (uint8_t *)R.mem;
    D.spins = m;
    const size_t sb = round_up(spin_bytes(&d, fmt), 256);
    D.rec = (islf_obs *)(m + sb);
    D.acc = (long long *)(m + sb + round_up((size_t)cap * sizeof(islf_obs), 256));
    build_tables(&d, D);
    D.Lx = d.Lx; D.Ly = d.Ly; D.Lz = d.Lz;
    D.C = (d.Lz + 7) / 8;
    D.K = (d.Lz + 15) / 16;
    D.Hp = 8 * D.K;
    D.RB = 2 * D.Hp;
    D.Wq = (d.Lz + 63) / 64;
    D.seam_reflect = d.ybc == ISLF_YBC_GAPBC;
    D.seam_invert = d.ybc != ISLF_YBC_PBC;
    D.key0 = (uint32_t)(d.seed & 0xFFFFFFFFull);
    D.key1 = (uint32_t)(d.seed >> 32);
    D.replica = d.replica;
    D.cap = cap;
    D.fmt = fmt;
    D.J = d.J; D.H = d.H; D.h1 = d.h1; D.hn = d.hn;
}

// ---------------------------------------------------------------------------
// device-side tables
// ---------------------------------------------------------------------------
static islf_status ensure_slots(islf_ctx *c, int n)
{
    if (n <= c->slot_capacity) return ISLF_OK;
    int cap = std::max(n, std::max(16, 2 * c->slot_capacity));
    RepDesc *nd = (RepDesc *)dev_alloc(c, sizeof(RepDesc) * cap);
    RepState *ns = (RepState *)dev_alloc(c, sizeof(RepState) * cap);
    if (!nd || !ns) {
        dev_free(c, nd);
        dev_free(c, ns);
        return fail(ISLF_ENOMEM, "cannot allocate replica tables for %d slots", cap);
    }
    HIP_TRY(launch_zero((unsigned long long *)ns, (long)(sizeof(RepState) * cap / 8), c->stream));
    if (c->d_state) {
        HIP_TRY(hipMemcpyAsync(ns, c->d_state, sizeof(RepState) * c->slot_capacity, hipMemcpyDeviceToDevice,
                               c->stream));
        HIP_TRY(hipMemcpyAsync(nd, c->d_desc, sizeof(RepDesc) * c->slot_capacity, hipMemcpyDeviceToDevice,
                               c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    dev_free(c, c->d_desc);
    dev_free(c, c->d_state);
    c->d_desc = nd;
    c->d_state = ns;
    c->slot_capacity = cap;
    c->graph_valid = false;
    return ISLF_OK;
}

static void free_plan(islf_ctx *c, Plan &p)
{
    dev_free(c, p.items);
    dev_free(c, p.first);
    p = Plan();
}

// Shares of a launch are tapered by dispatch rank (later workgroups get
// less) against the uneven progress of the workgroups resident on one CU
// (issue goes oldest first).  Measured on the 3 x 160x480x600 workload, by
// graph replay of the grouped batched form: bit-packed is fastest untapered
// (+1.2% over +-20%), int8 at +-10..30% (+0.5%).
static double tail_taper(int fmt)
{
    return fmt == ISLF_SPIN_BITPACK ? 0.0 : 0.1;
}
// a plain launch holds one replica: shorter launches, whose tails weigh more
constexpr double kPlainTaper = 0.2;
// the persistent launch has no second round of workgroups to fill a CU
// whose resident workgroups finish at different times: issue goes oldest
// first, and per-workgroup timestamps of a launch over three 46M lattices
// showed the workgroups of the first, second and third dispatch round (one
// per CU each) finishing equal shares after 19.6, 27 and 36 us.  Its shares
// therefore step down by dispatch round (grid and team barriers alike);
// 0.4 measured best or within noise of it (grid barriers: bit-packed 1,869
// against 1,812 untapered, int8 1,133 against 1,122; teams: int8 1,297
// against 1,152, bit-packed 1,653 against 1,614; 0 .. 0.7 tried)
constexpr double kPersistentTaper = 0.4;
// three concurrent groups: measured as fast as two and faster than four on
// every batch tried (3 x 160x480x600, 64 x 40x120x120, 96 uneven replicas);
// four group streams can share one of the process's four hardware queues
constexpr int kAutoGroups = 3;
constexpr int kMaxStreamGroups = 16;   // concurrent replica groups of the batched form (hardware queues per process)

// Splits the work into about `grid` runs of equal cost, one per workgroup:
// workgroup b gets items [first[b], first[b+1]).  The slab items are spread
// over the first min(grid, #slab) workgroups (so that a final launch of
// those workgroups covers them all); main tiles follow in order and fill
// every workgroup up to its share.  A main tile costs 4 units per x step and
// may be cut between steps; a slab tile costs 6 units (1.5 steps) per task
// per thread over its three row stages and is never cut.  The runs may be a
// part of a larger launch: run r is then the launch's run p0 + r of
// launch_grid, which sets its dispatch rank for the taper.  Returns the
// number of workgroups holding slab items.
static int partition_items(const std::vector<Entry> &slab, const std::vector<Entry> &main, int grid,
                           std::vector<Entry> &items, std::vector<int> &first, double taper, int p0 = 0,
                           int launch_grid = 0, int round = 0)
{
    auto slab_cost = [](const Entry &e) -> long long {
        const long long tasks = 6ll * e.y0 * e.nsteps;
        return 6 * ((tasks + kBlock - 1) / kBlock);
    };
    const long long ns = (long long)slab.size();
    long long W = 0, steps = 0;
    for (const Entry &e : slab) W += slab_cost(e);
    for (const Entry &e : main) steps += e.nsteps;
    W += 4 * steps;
    grid = (int)std::max(1ll, std::min((long long)grid, ns + steps));
    const long long gs = std::min<long long>(grid, ns);   // workgroups holding slab items
    items.clear();
    first.assign(1, 0);
    size_t mi = 0;   // next main tile and x offset inside it
    int off = 0;
    long long acc = 0;
    // cumulative cost targets: run r goes to the workgroup dispatched at rank
    // d(r) (the inverse of the kernel's XCD-contiguous mapping); later ranks
    // get smaller shares, weight 1 + a (1 - 2 u) at u = (d + 0.5) / grid
    const double a = taper;
    const long LG = launch_grid > 0 ? launch_grid : grid;
    std::vector<double> cum(grid + 1, 0.0);
    const long q = LG / 8, r8 = LG % 8;
    for (int r = 0; r < grid; ++r) {
        // the kernel gives XCD x (blocks x, x+8, ...) the runs from x*q + min(x, r8)
        const long rg = std::min<long>(p0 + r, LG - 1);
        long x, k;
        if (rg < r8 * (q + 1)) {
            x = rg / (q + 1);
            k = rg % (q + 1);
        } else {
            x = r8 + (rg - r8 * (q + 1)) / q;
            k = (rg - r8 * (q + 1)) % q;
        }
        const long d = x + 8 * k;
        // round > 0: a cooperative grid of `round` workgroups per dispatch
        // round (one per CU); the taper is a step per round
        const double u = round > 0 ? ((double)(d / round) + 0.5) / (double)((LG + round - 1) / round) : (d + 0.5) / LG;
        cum[r + 1] = cum[r] + 1.0 + a * (1.0 - 2.0 * u);
    }
    for (int b = 0; b < grid; ++b) {
        const long long target = (long long)((double)W * cum[b + 1] / cum[grid]);
        if (b < gs)
            for (long long k = b * ns / gs; k < (b + 1) * ns / gs; ++k) {
                items.push_back(slab[k]);
                acc += slab_cost(slab[k]);
            }
        while (mi < main.size() && (b == grid - 1 || target - acc >= 2)) {
            const Entry &e = main[mi];
            const int rem = e.nsteps - off;
            const int take = b == grid - 1 ? rem : (int)std::min<long long>(rem, std::max(1ll, (target - acc + 2) / 4));
            Entry piece = e;
            piece.x0 = e.x0 + off;
            piece.nsteps = take;
            items.push_back(piece);
            acc += 4ll * take;
            off += take;
            if (off == e.nsteps) {
                ++mi;
                off = 0;
            }
        }
        first.push_back((int)items.size());
        if (b + 1 >= gs && mi == main.size()) break;   // nothing left for later workgroups
    }
    return (int)gs;
}

static islf_status upload_plan(islf_ctx *c, Plan &p, const std::vector<Entry> &items, const std::vector<int> &first);

static islf_status build_plan(islf_ctx *c, Plan &p, const std::vector<Entry> &slab, const std::vector<Entry> &main,
                              int grid, double taper = -1.0, int round = 0)
{
    std::vector<Entry> items;
    std::vector<int> first;
    p.slab_grid = partition_items(slab, main, grid, items, first, taper < 0.0 ? tail_taper(c->fmt) : taper, 0, 0,
                                  round);
    return upload_plan(c, p, items, first);
}

static islf_status upload_plan(islf_ctx *c, Plan &p, const std::vector<Entry> &items, const std::vector<int> &first)
{
    p.grid = (int)first.size() - 1;
    if ((long)items.size() > p.items_cap) {
        dev_free(c, p.items);
        p.items_cap = std::max<long>((long)items.size(), 2 * p.items_cap);
        p.items = (Entry *)dev_alloc(c, sizeof(Entry) * p.items_cap);
        if (!p.items) return fail(ISLF_ENOMEM, "cannot allocate a launch plan");
    }
    if ((long)first.size() > p.first_cap) {
        dev_free(c, p.first);
        p.first_cap = std::max<long>((long)first.size(), 2 * p.first_cap);
        p.first = (int *)dev_alloc(c, sizeof(int) * p.first_cap);
        if (!p.first) return fail(ISLF_ENOMEM, "cannot allocate a launch plan");
    }
    if (!items.empty())
        HIP_TRY(hipMemcpyAsync(p.items, items.data(), sizeof(Entry) * items.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(p.first, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    p.valid = true;
    return ISLF_OK;
}

// Rebuilds the live list and the device descriptors after a change of
// membership or tiles; launch plans are rebuilt on their next use.
static islf_status sync_tables(islf_ctx *c)
{
    if (!c->dirty) return ISLF_OK;
    c->live.clear();
    const int n = (int)c->reps.size();
    for (int i = 0; i < n; ++i)
        if (c->reps[i].live) c->live.push_back(i);
    if ((int)c->live.size() > c->live_capacity) {
        dev_free(c, c->d_live);
        c->live_capacity = std::max<int>((int)c->live.size(), 2 * c->live_capacity);
        c->d_live = (int *)dev_alloc(c, sizeof(int) * c->live_capacity);
        if (!c->d_live) return fail(ISLF_ENOMEM, "cannot allocate live list");
    }
    if (!c->live.empty())
        HIP_TRY(hipMemcpyAsync(c->d_live, c->live.data(), sizeof(int) * c->live.size(), hipMemcpyHostToDevice, c->stream));
    for (int i : c->live)
        HIP_TRY(hipMemcpyAsync(c->d_desc + i, &c->reps[i].d, sizeof(RepDesc), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->batched.valid = false;
    c->persistent.valid = false;
    for (Plan &p : c->plain) p.valid = false;
    c->groups_valid = false;
    c->dirty = false;
    c->graph_valid = false;
    return ISLF_OK;
}

// The plans the context's execution form launches, built if needed.
static int num_groups(const islf_ctx *c)
{
    const int nl = (int)c->live.size();
    const int want = c->groups_req ? c->groups_req : kAutoGroups;
    return std::max(1, std::min(want, nl));
}

// Workgroups per A / B launch of a form: the override, else two per resident
// slot for one launch chain.  Concurrent groups share the resident slots:
// together they keep 3/2 workgroups per slot in flight, split evenly among
// the groups (the tail of one group's launch is filled by the others').
static int launch_grid(const islf_ctx *c, int exec)
{
    if (c->grid_override) return c->grid_override;
    const int G = exec == ISLF_EXEC_BATCHED ? num_groups(c) : 1;
    if (G == 1) return c->sweep_slots;
    return (int)std::max(64l, (3l * c->resident_slots + G) / (2l * G));
}

// Concurrent groups of the batched form: live replicas dealt to the group
// with the fewest sites so far (largest first), one launch plan per group
// (launch_grid: 3/2 x resident slots / groups workgroups, so that all groups
// together keep about 3/2 per slot in flight and each group's tail is filled
// by the others' launches), the groups' live lists on the device, and the
// groups' streams and fork / join events.
static islf_status prepare_groups(islf_ctx *c)
{
    islf_status st = sync_tables(c);
    if (st != ISLF_OK) return st;
    if (c->groups_valid) return ISLF_OK;
    const int G = num_groups(c);
    std::vector<int> order(c->live);
    auto sites = [&](int r) {
        const islf_replica_desc &d = c->reps[r].desc;
        return (long long)d.Lx * d.Ly * d.Lz;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sites(a) > sites(b); });
    std::vector<std::vector<int>> grp(G);
    std::vector<long long> load(G, 0);
    for (int r : order) {
        const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        grp[g].push_back(r);
        load[g] += sites(r);
    }
    std::vector<int> flat;
    c->group_off.assign(G, 0);
    c->group_len.assign(G, 0);
    for (int g = 0; g < G; ++g) {
        std::sort(grp[g].begin(), grp[g].end());
        c->group_off[g] = (int)flat.size();
        c->group_len[g] = (int)grp[g].size();
        flat.insert(flat.end(), grp[g].begin(), grp[g].end());
    }
    if ((int)flat.size() > c->group_live_cap) {
        dev_free(c, c->d_group_live);
        c->group_live_cap = std::max<int>((int)flat.size(), 2 * c->group_live_cap);
        c->d_group_live = (int *)dev_alloc(c, sizeof(int) * c->group_live_cap);
        if (!c->d_group_live) return fail(ISLF_ENOMEM, "cannot allocate group lists");
    }
    if (!flat.empty())
        HIP_TRY(hipMemcpyAsync(c->d_group_live, flat.data(), sizeof(int) * flat.size(), hipMemcpyHostToDevice,
                               c->stream));
    if ((int)c->group_plan.size() < G) c->group_plan.resize(G);
    for (int g = 0; g < G; ++g) {
        std::vector<Entry> S, M;
        for (int r : grp[g]) {
            S.insert(S.end(), c->reps[r].slab.begin(), c->reps[r].slab.end());
            M.insert(M.end(), c->reps[r].main.begin(), c->reps[r].main.end());
        }
        st = build_plan(c, c->group_plan[g], S, M, launch_grid(c, ISLF_EXEC_BATCHED), c->taper_override);
        if (st != ISLF_OK) return st;
    }
    while ((int)c->side_stream.size() < G) {
        hipStream_t sst = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&sst, hipStreamNonBlocking));
        c->side_stream.push_back(sst);
    }
    while ((int)c->side_event.size() < G + 1) {
        hipEvent_t ev = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        c->side_event.push_back(ev);
    }
    c->groups_valid = true;
    return ISLF_OK;
}

// The team form of the persistent plan: the grid's workgroups are dealt to
// the live replicas so that the largest number of sites per workgroup is as
// small as it can be (one each, then greedily), each replica's items are cut
// into equal-cost runs over its team, and the teams take contiguous plan
// slots (so a team's workgroups share an XCD where the team is small enough).
static islf_status build_team_plan(islf_ctx *c, int grid, double taper)
{
    const int nl = (int)c->live.size();
    std::vector<long long> sites(nl);
    for (int i = 0; i < nl; ++i) {
        const islf_replica_desc &d = c->reps[c->live[i]].desc;
        sites[i] = (long long)d.Lx * d.Ly * d.Lz;
    }
    // one workgroup each, then each further workgroup to the team with the
    // most sites per workgroup: the slowest team sets the launch's time
    std::vector<int> W(nl, 1);
    std::vector<std::pair<double, int>> heap;
    for (int i = 0; i < nl; ++i) heap.push_back({(double)sites[i], i});
    std::make_heap(heap.begin(), heap.end());
    for (int used = nl; used < grid; ++used) {
        std::pop_heap(heap.begin(), heap.end());
        const int i = heap.back().second;
        W[i] += 1;
        heap.back().first = (double)sites[i] / (double)W[i];
        std::push_heap(heap.begin(), heap.end());
    }
    std::vector<Entry> items;
    std::vector<int> first(1, 0);
    std::vector<TeamInfo> teams;
    for (int i = 0; i < nl; ++i) {
        const int r = c->live[i];
        std::vector<Entry> it;
        std::vector<int> fi;
        // the team's runs are the launch's runs first.size()-1 onwards: their
        // dispatch ranks in the launch set the taper
        partition_items(c->reps[r].slab, c->reps[r].main, W[i], it, fi, taper, (int)first.size() - 1, grid,
                        c->num_cu);
        const int n = (int)fi.size() - 1;
        const int off = (int)items.size();
        items.insert(items.end(), it.begin(), it.end());
        for (int b = 0; b < n; ++b) {
            first.push_back(off + fi[b + 1]);
            teams.push_back(TeamInfo{r, b, n, 0});
        }
    }
    if ((long)teams.size() > c->teams_cap) {
        dev_free(c, c->d_teams);
        c->teams_cap = std::max<long>((long)teams.size(), 2 * c->teams_cap);
        c->d_teams = (TeamInfo *)dev_alloc(c, sizeof(TeamInfo) * c->teams_cap);
        if (!c->d_teams) return fail(ISLF_ENOMEM, "cannot allocate team records");
    }
    if (c->slot_capacity > c->rsync_cap) {
        dev_free(c, c->d_rsync);
        c->rsync_cap = c->slot_capacity;
        c->d_rsync = (SyncLine *)dev_alloc(c, 2 * sizeof(SyncLine) * c->rsync_cap);
        if (!c->d_rsync) return fail(ISLF_ENOMEM, "cannot allocate team counters");
    }
    HIP_TRY(hipMemcpyAsync(c->d_teams, teams.data(), sizeof(TeamInfo) * teams.size(), hipMemcpyHostToDevice,
                           c->stream));
    c->persistent_teams = true;
    return upload_plan(c, c->persistent, items, first);
}

// Whether the persistent launch uses team barriers.  Automatic: teams for
// int8 spins or batches of 8 or more replicas, grid barriers for a few
// bit-packed replicas; measured (updates/ns, grid / team): 3 x 160x480x600
// bit-packed 1,780 / 1,562, int8 1,100 / 1,167; 64 x 40x120x120
// bit-packed 795 / 834, int8 646 / 779.  Teams need a workgroup for every
// live replica.
static bool use_teams(const islf_ctx *c, int grid)
{
    const int nl = (int)c->live.size();
    if (nl > grid) return false;
    if (c->team_mode >= 0) return c->team_mode == 1;
    return c->fmt == ISLF_SPIN_INT8 || nl >= 8;
}

static islf_status prepare_plans(islf_ctx *c, int exec)
{
    islf_status st = sync_tables(c);
    if (st != ISLF_OK) return st;
    auto lists = [&](const std::vector<int> &reps, std::vector<Entry> &S, std::vector<Entry> &M) {
        for (int r : reps) {
            S.insert(S.end(), c->reps[r].slab.begin(), c->reps[r].slab.end());
            M.insert(M.end(), c->reps[r].main.begin(), c->reps[r].main.end());
        }
    };
    if (c->live.empty()) return ISLF_OK;
    if (exec == ISLF_EXEC_BATCHED && num_groups(c) > 1) return prepare_groups(c);
    if (exec == ISLF_EXEC_BATCHED && !c->batched.valid) {
        std::vector<Entry> S, M;
        lists(c->live, S, M);
        return build_plan(c, c->batched, S, M, c->grid_override ? c->grid_override : c->sweep_slots,
                          c->taper_override);
    }
    if (exec == ISLF_EXEC_PERSISTENT && !c->persistent.valid) {
        std::vector<Entry> S, M;
        lists(c->live, S, M);
        const int grid = c->grid_override ? c->grid_override : c->persistent_grid;
        if (grid > c->persistent_bound)
            return fail(ISLF_ERANGE, "persistent grid %d exceeds the co-residency bound %d of this device", grid,
                        c->persistent_bound);
        // team plans taper by their launch-wide dispatch rounds too
        if (use_teams(c, grid))
            return build_team_plan(c, grid, c->taper_override >= 0.0 ? c->taper_override : kPersistentTaper);
        const double taper = c->taper_override >= 0.0 ? c->taper_override : kPersistentTaper;
        c->persistent_teams = false;
        return build_plan(c, c->persistent, S, M, grid, taper, c->num_cu);
    }
    if (exec == ISLF_EXEC_PLAIN) {
        if (c->plain.size() < c->reps.size()) c->plain.resize(c->reps.size());
        for (int r : c->live) {
            if (c->plain[r].valid) continue;
            std::vector<Entry> S, M;
            lists(std::vector<int>(1, r), S, M);
            st = build_plan(c, c->plain[r], S, M, c->grid_override ? c->grid_override : c->sweep_slots, kPlainTaper);
            if (st != ISLF_OK) return st;
        }
    }
    return ISLF_OK;
}

// init spins + initial observables of slot i (synchronises)
static islf_status init_replica(islf_ctx *c, int i, int mode, const int8_t *host_staged)
{
    Replica &R = c->reps[i];
    HIP_TRY(hipMemcpyAsync(c->d_desc + i, &R.d, sizeof(RepDesc), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(launch_zero((unsigned long long *)R.d.acc, 2 * kAccSlots * 4, c->stream));
    HIP_TRY(launch_init(c->fmt, c->d_desc, i, mode, host_staged, c->stream));
    const size_t N = (size_t)R.desc.Lx * R.desc.Ly * R.desc.Lz;
    int8_t *tmp = (int8_t *)dev_alloc(c, N);
    if (!tmp) return fail(ISLF_ENOMEM, "cannot allocate %zu bytes of staging", N);
    hipError_t e = launch_export(c->d_desc, i, (long)R.desc.Lx * R.desc.Ly, tmp, c->stream);
    if (e == hipSuccess)
        e = launch_recompute(c->d_desc, i, (long)R.desc.Lx * R.desc.Ly, tmp, c->d_scratch, c->stream);
    if (e == hipSuccess) e = launch_set_state(c->d_state, i, c->d_scratch, 0u, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dev_free(c, tmp);
    if (e != hipSuccess) return fail(ISLF_EDEVICE, "replica init failed: %s", hipGetErrorString(e));
    R.t_host = 0;
    return ISLF_OK;
}

static islf_status add_replica(islf_ctx *c, const islf_replica_desc *desc, int *slot_out)
{
    islf_status st = validate(desc);
    if (st != ISLF_OK) return st;
    int slot = -1;
    for (int i = 0; i < (int)c->reps.size(); ++i)
        if (!c->reps[i].live) {
            slot = i;
            break;
        }
    if (slot < 0) {
        slot = (int)c->reps.size();
        c->reps.emplace_back();
    }
    st = ensure_slots(c, (int)c->reps.size());
    if (st != ISLF_OK) return st;
    Replica &R = c->reps[slot];
    R.desc = *desc;
    const size_t bytes = replica_bytes(desc, c->fmt, c->cap);
    if (R.mem && R.mem_bytes < bytes) {
        dev_free(c, R.mem);
        R.mem = nullptr;
    }
    if (!R.mem) {
        R.mem = dev_alloc(c, bytes);
        if (!R.mem) return fail(ISLF_ENOMEM, "cannot allocate %zu device bytes for a replica", bytes);
        R.mem_bytes = bytes;
    }
    R.tile = default_tile(desc, c->fmt);
    fill_desc(R, c->fmt, c->cap);
    build_work(R, slot, c->fmt);
    const int mode = desc->init == ISLF_INIT_HOST ? ISLF_INIT_UP : desc->init;
    st = init_replica(c, slot, mode, nullptr);
    if (st != ISLF_OK) return st;
    R.live = true;
    c->dirty = true;
    *slot_out = slot;
    return ISLF_OK;
}

static void destroy_graphs(islf_ctx *c)
{
    for (hipGraphExec_t ex : c->graph_execs) (void)hipGraphExecDestroy(ex);
    for (hipGraph_t g : c->graphs) (void)hipGraphDestroy(g);
    c->graph_execs.clear();
    c->graphs.clear();
    c->graph_valid = false;
}

static void destroy_ctx(islf_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    destroy_graphs(c);
    for (auto &R : c->reps) dev_free(c, R.mem);
    dev_free(c, c->d_desc);
    dev_free(c, c->d_state);
    dev_free(c, c->d_sync);
    dev_free(c, c->d_teams);
    dev_free(c, c->d_rsync);
    dev_free(c, c->d_scratch);
    dev_free(c, c->d_live);
    free_plan(c, c->batched);
    free_plan(c, c->persistent);
    for (Plan &p : c->plain) free_plan(c, p);
    for (Plan &p : c->group_plan) free_plan(c, p);
    dev_free(c, c->d_group_live);
    for (hipStream_t sst : c->side_stream) (void)hipStreamDestroy(sst);
    for (hipEvent_t ev : c->side_event) (void)hipEventDestroy(ev);
    delete c;
}

// Workgroups of a 256-thread kernel that can be resident on one CU at once,
// the smaller of the runtime's occupancy answer and a count from the
// kernel's own resources: a workgroup is four wave64s, one per SIMD, so a
// SIMD's 512 VGPRs per lane (allocated in granules of 8) bound the
// workgroups per CU, and so do the CU's thread slots and LDS.
static int coresident_per_cu(const void *kernel, const hipDeviceProp_t &prop)
{
    int rt = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&rt, kernel, kBlock, 0) != hipSuccess || rt < 1) rt = 1;
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, kernel) != hipSuccess) return rt;
    int per_cu = rt;
    const int vgprs = std::max(1, (a.numRegs + 7) / 8 * 8);
    per_cu = std::min(per_cu, 512 / vgprs);
    if (prop.maxThreadsPerMultiProcessor > 0) per_cu = std::min(per_cu, prop.maxThreadsPerMultiProcessor / kBlock);
    if (a.sharedSizeBytes > 0 && prop.maxSharedMemoryPerMultiProcessor > 0)
        per_cu = std::min(per_cu, (int)(prop.maxSharedMemoryPerMultiProcessor / a.sharedSizeBytes));
    return std::max(1, per_cu);
}

// ---------------------------------------------------------------------------
// public API
// ---------------------------------------------------------------------------
extern "C" islf_status islf_create_with_allocator(const islf_replica_desc *reps, int32_t n_reps,
                                                  int32_t spin_format, uint32_t obs_capacity,
                                                  void *hip_stream, islf_alloc_fn alloc,
                                                  islf_free_fn free_fn, void *user, islf_ctx **out)
{
    if (!out) return fail(ISLF_EINVAL, "NULL output pointer");
    *out = nullptr;
    if (!reps || n_reps < 1) return fail(ISLF_EINVAL, "need at least one replica");
    if (spin_format != ISLF_SPIN_INT8 && spin_format != ISLF_SPIN_BITPACK)
        return fail(ISLF_EINVAL, "invalid spin format %d", spin_format);
    if (obs_capacity < 1) return fail(ISLF_EINVAL, "obs_capacity must be >= 1");
    if ((alloc == nullptr) != (free_fn == nullptr)) return fail(ISLF_EINVAL, "give both alloc and free or neither");
    for (int i = 0; i < n_reps; ++i) {
        islf_status st = validate(&reps[i]);
        if (st != ISLF_OK) return st;
    }
    islf_ctx *c = new islf_ctx();
    c->fmt = spin_format;
    c->cap = obs_capacity;
    c->stream = (hipStream_t)hip_stream;
    c->alloc = alloc;
    c->free_fn = free_fn;
    c->user = user;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete c;
        return fail(ISLF_EDEVICE, "no HIP device");
    }
    c->num_cu = prop.multiProcessorCount;
    int per_cu_sweep = 0;
    if (sweep_blocks_per_cu(spin_format, &per_cu_sweep) != hipSuccess || per_cu_sweep < 1) per_cu_sweep = 1;
    // two workgroups per resident slot: measured faster than one (a single
    // round leaves slots idle while the last workgroups finish)
    c->resident_slots = c->num_cu * per_cu_sweep;
    c->sweep_slots = 2 * c->resident_slots;
    // both forms of the persistent kernel (grid and team barriers) launch on
    // the same grid: the bound is the smaller of the two
    const int per_cu = std::min(coresident_per_cu(persistent_kernel(spin_format), prop),
                                coresident_per_cu(persistent_teams_kernel(spin_format), prop));
    c->persistent_bound = std::min(c->num_cu * per_cu, kBarrierGroup * kMaxGroups);
    // one slot per CU stays free by default: at the full occupancy the
    // runtime reported for an earlier build of the int8 kernel (7 workgroups
    // per CU at 72 VGPRs) a cooperative launch was accepted but its workgroups
    // were not all resident at once, and the grid barrier's bounded wait
    // expired
    const int per_cu_p = per_cu > 1 ? per_cu - 1 : 1;
    c->persistent_grid = std::min(c->num_cu * per_cu_p, c->persistent_bound);
    if (noalloc_scratch(&c->noalloc_scratch) != hipSuccess) {
        delete c;
        return fail(ISLF_EDEVICE, "cannot look up the means scratch array on device %d", dev);
    }
    c->d_sync = (GridSync *)dev_alloc(c, sizeof(GridSync));
    c->d_scratch = (unsigned long long *)dev_alloc(c, 64 * sizeof(unsigned long long));
    if (!c->d_sync || !c->d_scratch) {
        destroy_ctx(c);
        return fail(ISLF_ENOMEM, "cannot allocate context buffers");
    }
    if (launch_zero((unsigned long long *)c->d_sync, sizeof(GridSync) / 8, c->stream) != hipSuccess) {
        destroy_ctx(c);
        return fail(ISLF_EDEVICE, "cannot clear sync words");
    }
    for (int i = 0; i < n_reps; ++i) {
        int slot;
        islf_status st = add_replica(c, &reps[i], &slot);
        if (st != ISLF_OK) {
            std::string keep = g_err;
            destroy_ctx(c);
            g_err = keep;
            return st;
        }
    }
    islf_status st = sync_tables(c);
    if (st != ISLF_OK) {
        std::string keep = g_err;
        destroy_ctx(c);
        g_err = keep;
        return st;
    }
    *out = c;
    return ISLF_OK;
}

extern "C" islf_status islf_create(const islf_replica_desc *reps, int32_t n_reps, int32_t spin_format,
                                   uint32_t obs_capacity, void *hip_stream, islf_ctx **out)
{
    return islf_create_with_allocator(reps, n_reps, spin_format, obs_capacity, hip_stream, nullptr, nullptr,
                                      nullptr, out);
}

extern "C" islf_status islf_destroy(islf_ctx *ctx)
{
    if (!ctx) return fail(ISLF_EINVAL, "NULL context");
    destroy_ctx(ctx);
    return ISLF_OK;
}

extern "C" islf_status islf_num_replicas(const islf_ctx *ctx, int32_t *n)
{
    if (!ctx || !n) return fail(ISLF_EINVAL, "NULL argument");
    *n = (int32_t)ctx->reps.size();
    return ISLF_OK;
}

static islf_status check_rep(const islf_ctx *ctx, int32_t rep)
{
    if (!ctx) return fail(ISLF_EINVAL, "NULL context");
    if (rep < 0 || rep >= (int32_t)ctx->reps.size() || !ctx->reps[rep].live)
        return fail(ISLF_ERANGE, "replica %d is not live", rep);
    return ISLF_OK;
}

extern "C" islf_status islf_get_desc(const islf_ctx *ctx, int32_t rep, islf_replica_desc *out)
{
    islf_status st = check_rep(ctx, rep);
    if (st != ISLF_OK) return st;
    if (!out) return fail(ISLF_EINVAL, "NULL output");
    *out = ctx->reps[rep].desc;
    return ISLF_OK;
}

extern "C" islf_status islf_set_spins(islf_ctx *ctx, int32_t rep, const int8_t *host, size_t n)
{
    islf_status st = check_rep(ctx, rep);
    if (st != ISLF_OK) return st;
    Replica &R = ctx->reps[rep];
    const size_t N = (size_t)R.desc.Lx * R.desc.Ly * R.desc.Lz;
    if (!host || n != N) return fail(ISLF_EINVAL, "expected %zu spins, got %zu", N, n);
    if (R.t_host != 0 && !R.failed)
        return fail(ISLF_ESTATE, "set_spins is only valid before the first sweep (or after a failed launch)");
    // +1 and -1 are the bytes 0x01 and 0xFF: (byte + 1) & 0xFD is 0 exactly for
    // them (a branch-free pass the compiler vectorises; the index of a bad
    // value is looked up only when there is one)
    uint8_t bad = 0;
    const uint8_t *hb = (const uint8_t *)host;
    for (size_t i = 0; i < n; ++i) bad |= (uint8_t)(hb[i] + 1u) & 0xFDu;
    if (bad)
        for (size_t i = 0; i < n; ++i)
            if (host[i] != 1 && host[i] != -1) return fail(ISLF_EINVAL, "spin %zu is %d, not +-1", i, (int)host[i]);
    int8_t *staged = (int8_t *)dev_alloc(ctx, N);
    if (!staged) return fail(ISLF_ENOMEM, "cannot allocate staging");
    hipError_t e = hipMemcpyAsync(staged, host, N, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        dev_free(ctx, staged);
        return fail(ISLF_EDEVICE, "copy of host spins failed: %s", hipGetErrorString(e));
    }
    st = init_replica(ctx, rep, 3, staged);
    dev_free(ctx, staged);
    if (st == ISLF_OK && R.failed) {
        R.failed = false;
        ctx->graph_valid = false;
    }
    return st;
}

extern "C" islf_status islf_get_spins(islf_ctx *ctx, int32_t rep, int8_t *host, size_t n)
{
    islf_status st = check_rep(ctx, rep);
    if (st != ISLF_OK) return st;
    Replica &R = ctx->reps[rep];
    const size_t N = (size_t)R.desc.Lx * R.desc.Ly * R.desc.Lz;
    if (!host || n != N) return fail(ISLF_EINVAL, "expected %zu spins, got %zu", N, n);
    st = check_intact(ctx, rep);
    if (st != ISLF_OK) return st;
    int8_t *tmp = (int8_t *)dev_alloc(ctx, N);
    if (!tmp) return fail(ISLF_ENOMEM, "cannot allocate staging");
    hipError_t e = launch_export(ctx->d_desc, rep, (long)R.desc.Lx * R.desc.Ly, tmp, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host, tmp, N, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    dev_free(ctx, tmp);
    if (e != hipSuccess) return fail(ISLF_EDEVICE, "get_spins failed: %s", hipGetErrorString(e));
    return ISLF_OK;
}

extern "C" islf_status islf_set_exec(islf_ctx *ctx, int32_t mode)
{
    if (!ctx) return fail(ISLF_EINVAL, "NULL context");
    if (mode < ISLF_EXEC_PLAIN || mode > ISLF_EXEC_PERSISTENT) return fail(ISLF_EINVAL, "invalid exec mode %d", mode);
    ctx->exec = mode;
    return ISLF_OK;
}

// Enqueues n >= 1 sweeps of the replicas in the device list dl (nl ids) over
// a plan: A(s) B(s) for each sweep, then F and the closing fold.  Optional
// events bracket each launch (A and B of sweep s at ev[4s..4s+3], F + fold
// at ev[4n], ev[4n+1]).
static hipError_t enqueue_plan(islf_ctx *c, const Plan &p, const int *dl, int nl, uint32_t n,
                               hipEvent_t *ev = nullptr, hipStream_t strm = nullptr)
{
    if (!strm) strm = c->stream;
    hipError_t e = hipSuccess;
    auto mark = [&](size_t i) {
        if (ev && e == hipSuccess) e = hipEventRecord(ev[i], strm);
    };
    for (uint32_t s = 0; s < n && e == hipSuccess; ++s) {
        mark(4 * (size_t)s);
        if (e == hipSuccess)
            e = launch_sweep(c->fmt, KIND_A, c->d_desc, c->d_state, p.items, p.first, p.grid, dl, nl, s,
                             s ? FLAG_PREV : 0u, strm);
        mark(4 * (size_t)s + 1);
        mark(4 * (size_t)s + 2);
        if (e == hipSuccess)
            e = launch_sweep(c->fmt, KIND_B, c->d_desc, c->d_state, p.items, p.first, p.grid, dl, nl, s,
                             s ? FLAG_FOLD : 0u, strm);
        mark(4 * (size_t)s + 3);
    }
    mark(4 * (size_t)n);
    if (e == hipSuccess)
        e = launch_sweep(c->fmt, KIND_F, c->d_desc, c->d_state, p.items, p.first, p.slab_grid, dl, nl, n - 1, 0u,
                         strm);
    if (e == hipSuccess) e = launch_fold(c->d_desc, c->d_state, dl, nl, n - 1, n, strm);
    mark(4 * (size_t)n + 1);
    return e;
}

// Enqueues n sweeps in the context's execution form (plans prepared, no
// checks, no sync).
// Concurrent groups: group g issues on side stream g, a stream the context
// creates, group 0 included.  Fork: every side stream waits for the work
// issued before on the context's stream; join: the context's stream waits for
// every side stream.  The context's own stream (the caller's) carries no group
// work: the runtime maps streams onto a few hardware queues, and with the
// caller's stream carrying group 0, some contexts of a process ran a batch at
// 1,700 instead of 2,400 updates/ns (bit-packed), as when two groups share a
// queue and serialise; with the context's own streams for every group they
// did not.  An ungrouped context issues on its own stream.
static hipStream_t group_stream(const islf_ctx *c, int g, int G)
{
    return G > 1 ? c->side_stream[g] : c->stream;
}

static hipError_t fork_groups(islf_ctx *c, int G)
{
    hipError_t e = hipEventRecord(c->side_event[0], c->stream);
    for (int g = 0; g < G && e == hipSuccess; ++g) e = hipStreamWaitEvent(c->side_stream[g], c->side_event[0], 0);
    return e;
}

static hipError_t join_groups(islf_ctx *c, int G)
{
    hipError_t e = hipSuccess;
    for (int g = 0; g < G && e == hipSuccess; ++g) {
        e = hipEventRecord(c->side_event[g + 1], c->side_stream[g]);
        if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->side_event[g + 1], 0);
    }
    return e;
}

static hipError_t enqueue_group(islf_ctx *c, int g, uint32_t n)
{
    return enqueue_plan(c, c->group_plan[g], c->d_group_live + c->group_off[g], c->group_len[g], n, nullptr,
                        c->side_stream[g]);
}

static islf_status enqueue_sweeps(islf_ctx *c, uint32_t n)
{
    const int nl = (int)c->live.size();
    if (nl == 0 || n == 0) return ISLF_OK;
    if (c->exec == ISLF_EXEC_PERSISTENT) {
        const Plan &p = c->persistent;
        hipError_t e = c->persistent_teams
                           ? launch_persistent_teams(c->fmt, c->d_desc, c->d_state, p.items, p.first, c->d_teams, n,
                                                     c->d_sync, c->d_rsync, c->rsync_cap, p.grid, c->stream)
                           : launch_persistent(c->fmt, c->d_desc, c->d_state, p.items, p.first, c->d_live, nl, n,
                                               c->d_sync, p.grid, c->stream);
        if (e != hipSuccess) return fail(ISLF_EDEVICE, "persistent launch failed: %s", hipGetErrorString(e));
        return ISLF_OK;
    }
    if (c->exec == ISLF_EXEC_BATCHED && num_groups(c) > 1) {
        const int G = num_groups(c);
        HIP_TRY(fork_groups(c, G));
        for (int g = 0; g < G; ++g) HIP_TRY(enqueue_group(c, g, n));
        HIP_TRY(join_groups(c, G));
        return ISLF_OK;
    }
    if (c->exec == ISLF_EXEC_BATCHED) {
        HIP_TRY(enqueue_plan(c, c->batched, c->d_live, nl, n));
        return ISLF_OK;
    }
    // plain: one lattice per launch; replica r's fold list is its entry in d_live
    for (uint32_t s = 0; s < n; ++s)
        for (int k = 0; k < 2; ++k)
            for (int li = 0; li < nl; ++li) {
                const Plan &p = c->plain[c->live[li]];
                HIP_TRY(launch_sweep(c->fmt, k, c->d_desc, c->d_state, p.items, p.first, p.grid, c->d_live + li, 1,
                                     s, s ? (k == 0 ? FLAG_PREV : FLAG_FOLD) : 0u, c->stream));
            }
    for (int li = 0; li < nl; ++li) {
        const Plan &p = c->plain[c->live[li]];
        HIP_TRY(launch_sweep(c->fmt, KIND_F, c->d_desc, c->d_state, p.items, p.first, p.slab_grid, c->d_live + li,
                             1, n - 1, 0u, c->stream));
    }
    HIP_TRY(launch_fold(c->d_desc, c->d_state, c->d_live, nl, n - 1, n, c->stream));
    return ISLF_OK;
}

// Reads the persistent kernel's error word (synchronises).  A raised word
// means a launch gave up at a grid barrier and left its sweeps half done, so
// every live replica is marked failed (its calls return ESTATE until
// islf_set_spins restarts it or it is retired); the word is then cleared so
// that later launches can run.
static islf_status check_device_error(islf_ctx *c)
{
    unsigned long long err = 0;
    HIP_TRY(hipMemcpyAsync(&err, &c->d_sync->error.v, sizeof err, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (err) {
        for (int r : c->live) c->reps[r].failed = true;
        c->graph_valid = false;
        HIP_TRY(launch_zero((unsigned long long *)&c->d_sync->error, 16, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        return fail(ISLF_EDEVICE, "a persistent-kernel grid barrier gave up (its workgroups were not all resident at "
                                  "once, or the wait was cut short); every live replica is marked failed");
    }
    return ISLF_OK;
}

// A live replica whose chain is intact: checks the device error word, then
// the replica's failed mark.
static islf_status check_intact(islf_ctx *c, int rep)
{
    islf_status st = check_device_error(c);
    if (st != ISLF_OK) return st;
    if (c->reps[rep].failed)
        return fail(ISLF_ESTATE, "replica %d was cut short by a failed persistent launch (restart it with "
                                 "islf_set_spins or retire it)", rep);
    return ISLF_OK;
}

static islf_status check_none_failed(const islf_ctx *c)
{
    for (int r : c->live)
        if (c->reps[r].failed)
            return fail(ISLF_ESTATE, "replica %d was cut short by a failed persistent launch (restart it with "
                                     "islf_set_spins or retire it)", r);
    return ISLF_OK;
}

static islf_status check_sweep_range(islf_ctx *c, uint64_t n)
{
    for (int r : c->live)
        if (c->reps[r].t_host + n > 0xFFFFFFFFull)
            return fail(ISLF_ERANGE, "replica %d would pass 2^32-1 sweeps", r);
    return ISLF_OK;
}

extern "C" islf_status islf_sweep(islf_ctx *ctx, uint32_t n_sweeps)
{
    if (!ctx) return fail(ISLF_EINVAL, "NULL context");
    islf_status st = check_none_failed(ctx);
    if (st != ISLF_OK) return st;
    st = prepare_plans(ctx, ctx->exec);
    if (st != ISLF_OK) return st;
    st = check_sweep_range(ctx, n_sweeps);
    if (st != ISLF_OK) return st;
    st = enqueue_sweeps(ctx, n_sweeps);
    if (st != ISLF_OK) return st;
    for (int r : ctx->live) ctx->reps[r].t_host += n_sweeps;
    return ISLF_OK;
}

extern "C" islf_status islf_sweep_count(islf_ctx *ctx, int32_t rep, uint64_t *t)
{
    islf_status st = check_rep(ctx, rep);
    if (st != ISLF_OK) return st;
    if (!t) return fail(ISLF_EINVAL, "NULL output");
    st = check_intact(ctx, rep);
    if (st != ISLF_OK) return st;
    RepState s;
    HIP_TRY(hipMemcpyAsync(&s, ctx->d_state + rep, sizeof s, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (s.t != (uint32_t)ctx->reps[rep].t_host)
        return fail(ISLF_EDEVICE, "device sweep counter %u != issued %llu", s.t,
                    (unsigned long long)ctx->reps[rep].t_host);
    *t = s.t;
    return ISLF_OK;
}

static islf_status check_records(islf_ctx *c, int rep, uint64_t first, uint32_t count)
{
    const uint64_t t = c->reps[rep].t_host;
    if (count == 0) return fail(ISLF_EINVAL, "count must be >= 1");
    if (first + count > t) return fail(ISLF_ERANGE, "records up to sweep %llu requested, %llu run",
                                       (unsigned long long)(first + count), (unsigned long long)t);
    if (t > c->cap && first < t - c->cap)
        return fail(ISLF_ERANGE, "record %llu has left the ring (capacity %u)", (unsigned long long)first, c->cap);
    return ISLF_OK;
}

extern "C" islf_status islf_measure(islf_ctx *ctx, int32_t rep, uint64_t first, uint32_t count, islf_obs *out)
{
    islf_status st = check_rep(ctx, rep);
    if (st != ISLF_OK) return st;
    if (!out) return fail(ISLF_EINVAL, "NULL output");
    st = check_records(ctx, rep, first, count);
    if (st != ISLF_OK) return st;
    st = check_intact(ctx, rep);
    if (st != ISLF_OK) return st;
    const Replica &R = ctx->reps[rep];
    uint32_t done = 0;
    while (done < count) {
        const uint32_t slot = (uint32_t)((first + done) % ctx->cap);
        const uint32_t n = std::min<uint32_t>(count - done, ctx->cap - slot);
        HIP_TRY(hipMemcpyAsync(out + done, R.d.rec + slot, n * sizeof(islf_obs), hipMemcpyDeviceToHost, ctx->stream));
        done += n;
    }
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return ISLF_OK;
}

extern "C" islf_status islf_recompute(islf_ctx *ctx, int32_t rep, islf_obs *out)
{
    islf_status st = check_rep(ctx, rep);
    if (st != ISLF_OK) return st;
    if (!out) return fail(ISLF_EINVAL, "NULL output");
    st = check_intact(ctx, rep);
    if (st != ISLF_OK) return st;
    const Replica &R = ctx->reps[rep];
    const size_t N = (size_t)R.desc.Lx * R.desc.Ly * R.desc.Lz;
    int8_t *tmp = (int8_t *)dev_alloc(ctx, N);
    if (!tmp) return fail(ISLF_ENOMEM, "cannot allocate staging");
    unsigned long long h[4];
    hipError_t e = launch_export(ctx->d_desc, rep, (long)R.desc.Lx * R.desc.Ly, tmp, ctx->stream);
    if (e == hipSuccess)
        e = launch_recompute(ctx->d_desc, rep, (long)R.desc.Lx * R.desc.Ly, tmp, ctx->d_scratch, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h, ctx->d_scratch, sizeof h, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    dev_free(ctx, tmp);
    if (e != hipSuccess) return fail(ISLF_EDEVICE, "recompute failed: %s", hipGetErrorString(e));
    out->B = (int64_t)h[0];
    out->M = (int64_t)h[1];
    out->M1 = (int64_t)h[2];
    out->Mn = (int64_t)h[3];
    return ISLF_OK;
}

extern "C" islf_status islf_record_energy(islf_ctx *ctx, int32_t rep, uint64_t first, uint32_t count,
                                          double *out)
{
    islf_status st = check_rep(ctx, rep);
    if (st != ISLF_OK) return st;
    if (!out) return fail(ISLF_EINVAL, "NULL output");
    st = check_records(ctx, rep, first, count);
    if (st != ISLF_OK) return st;
    st = check_intact(ctx, rep);
    if (st != ISLF_OK) return st;
    const Replica &R = ctx->reps[rep];
    double *tmp = (double *)dev_alloc(ctx, sizeof(double) * count);
    if (!tmp) return fail(ISLF_ENOMEM, "cannot allocate staging");
    hipError_t e = launch_energy(R.d.rec, ctx->cap, first, count, R.desc.J, R.desc.H, R.desc.h1, R.desc.hn, tmp,
                                 ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, sizeof(double) * count, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    dev_free(ctx, tmp);
    if (e != hipSuccess) return fail(ISLF_EDEVICE, "energy failed: %s", hipGetErrorString(e));
    return ISLF_OK;
}

extern "C" islf_status islf_means(islf_ctx *ctx, uint64_t first, uint32_t count, double *out)
{
    if (!ctx || !out) return fail(ISLF_EINVAL, "NULL argument");
    islf_status st = sync_tables(ctx);
    if (st != ISLF_OK) return st;
    const int n = (int)ctx->reps.size();
    for (int r = 0; r < n; ++r) {
        if (!ctx->reps[r].live) continue;
        st = check_records(ctx, r, first, count);
        if (st != ISLF_OK) return st;
    }
    st = check_device_error(ctx);
    if (st != ISLF_OK) return st;
    st = check_none_failed(ctx);
    if (st != ISLF_OK) return st;
    // live replicas only; dead slots report NaN
    const int nl = (int)ctx->live.size();
    std::vector<double> tmp_h(5 * (size_t)std::max(nl, 1));
    double *tmp = (double *)dev_alloc(ctx, sizeof(double) * 5 * std::max(nl, 1));
    if (!tmp) return fail(ISLF_ENOMEM, "cannot allocate staging");
    hipError_t e = hipSuccess;
    if (nl > 0) e = launch_means(ctx->d_desc, ctx->d_live, nl, first, count, tmp, ctx->stream);
    if (e == hipSuccess && nl > 0)
        e = hipMemcpyAsync(tmp_h.data(), tmp, sizeof(double) * 5 * nl, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    dev_free(ctx, tmp);
    if (e != hipSuccess) return fail(ISLF_EDEVICE, "means failed: %s", hipGetErrorString(e));
    for (int r = 0; r < n; ++r)
        for (int k = 0; k < 5; ++k) out[5 * r + k] = NAN;
    for (int i = 0; i < nl; ++i)
        for (int k = 0; k < 5; ++k) out[5 * ctx->live[i] + k] = tmp_h[5 * i + k];
    return ISLF_OK;
}

// Host FP64 energies of records (Sec. II.A Eq. 1), in the order the header
// states; plain C arithmetic (the library is built without FMA contraction).
extern "C" islf_status islf_energy(const islf_replica_desc *desc, const islf_obs *obs, size_t n, double *E_out)
{
    if (!desc) return fail(ISLF_EINVAL, "NULL replica descriptor");
    if (n > 0 && (!obs || !E_out)) return fail(ISLF_EINVAL, "NULL records or output");
    const double J = desc->J, H = desc->H, h1 = desc->h1, hn = desc->hn;
    if (!isfinite(J) || !isfinite(H) || !isfinite(h1) || !isfinite(hn))
        return fail(ISLF_EINVAL, "J, H, h1, hn must be finite");
    for (size_t k = 0; k < n; ++k) {
        double e = -J * (double)obs[k].B;
        e = e - H * (double)obs[k].M;
        e = e - h1 * (double)obs[k].M1;
        e = e - hn * (double)obs[k].Mn;
        E_out[k] = e;
    }
    return ISLF_OK;
}

// The means of islf_means with the kernel's output in the device's scratch
// array instead of a staging allocation; the per-replica results are copied
// to the front of out and moved to their slots from the back (slot ids of
// live replicas are ascending and never below their rank, so no result is
// overwritten before it is moved).
extern "C" islf_status islf_means_noalloc(islf_ctx *ctx, uint64_t first, uint32_t count, double *out)
{
    if (!ctx || !out) return fail(ISLF_EINVAL, "NULL argument");
    if (ctx->dirty)
        return fail(ISLF_ESTATE, "replica tables are not current (after islf_set_tile, sweep or call islf_means once)");
    const int n = (int)ctx->reps.size();
    const int nl = (int)ctx->live.size();
    if (nl > kNoAllocMaxReps)
        return fail(ISLF_ERANGE, "%d live replicas exceed the %d the allocation-free means serve per call", nl,
                    kNoAllocMaxReps);
    islf_status st;
    for (int r : ctx->live) {
        st = check_records(ctx, r, first, count);
        if (st != ISLF_OK) return st;
    }
    st = check_device_error(ctx);
    if (st != ISLF_OK) return st;
    st = check_none_failed(ctx);
    if (st != ISLF_OK) return st;
    if (nl > 0) {
        HIP_TRY(launch_means(ctx->d_desc, ctx->d_live, nl, first, count, ctx->noalloc_scratch, ctx->stream));
        HIP_TRY(hipMemcpyAsync(out, ctx->noalloc_scratch, sizeof(double) * 5 * nl, hipMemcpyDeviceToHost,
                               ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    for (int i = nl - 1; i >= 0; --i) {
        const int r = ctx->live[i];
        if (r != i)
            for (int k = 0; k < 5; ++k) out[5 * r + k] = out[5 * i + k];
    }
    int li = 0;
    for (int r = 0; r < n; ++r) {
        if (li < nl && ctx->live[li] == r) {
            ++li;
            continue;
        }
        for (int k = 0; k < 5; ++k) out[5 * r + k] = NAN;
    }
    return ISLF_OK;
}

// Host FP64 cumulative trapezoid (Eq. 9 / Eq. 22 over the field, Eq. 19 over
// beta), left to right.
extern "C" islf_status islf_integrate(const double *h, const double *mean_M1, const double *mean_Mn, int32_t n,
                                      double c1, double cn, double norm, double *cumulative_out)
{
    if (!h || !mean_M1 || !mean_Mn || !cumulative_out) return fail(ISLF_EINVAL, "NULL argument");
    if (n < 1) return fail(ISLF_EINVAL, "need n >= 1 points");
    double g_prev = norm * (c1 * mean_M1[0] + cn * mean_Mn[0]);
    double acc = 0.0;
    cumulative_out[0] = 0.0;
    for (int32_t r = 1; r < n; ++r) {
        const double g = norm * (c1 * mean_M1[r] + cn * mean_Mn[r]);
        const double step = 0.5 * (h[r] - h[r - 1]);
        acc = acc + step * (g_prev + g);
        cumulative_out[r] = acc;
        g_prev = g;
    }
    return ISLF_OK;
}

extern "C" islf_status islf_integrate_device(const double *h, const double *m1, const double *mn, int32_t n,
                                             double c1, double cn, double norm, double *out, void *hip_stream)
{
    if (!h || !m1 || !mn || !out) return fail(ISLF_EINVAL, "NULL argument");
    if (n < 1) return fail(ISLF_EINVAL, "need n >= 1 points");
    HIP_TRY(launch_integrate(h, m1, mn, n, c1, cn, norm, out, (hipStream_t)hip_stream));
    return ISLF_OK;
}

extern "C" islf_status islf_footprint_bytes(const islf_replica_desc *desc, int32_t spin_format,
                                            uint32_t obs_capacity, uint64_t *bytes)
{
    if (!bytes) return fail(ISLF_EINVAL, "NULL output");
    islf_status st = validate(desc);
    if (st != ISLF_OK) return st;
    if (spin_format != ISLF_SPIN_INT8 && spin_format != ISLF_SPIN_BITPACK)
        return fail(ISLF_EINVAL, "invalid spin format %d", spin_format);
    Replica R;
    R.desc = *desc;
    R.tile = default_tile(desc, spin_format);
    build_work(R, 0, spin_format);
    *bytes = replica_bytes(desc, spin_format, obs_capacity) + sizeof(Entry) * (R.main.size() + R.slab.size()) +
             sizeof(RepDesc) + sizeof(RepState);
    return ISLF_OK;
}

extern "C" islf_status islf_plan_preview(const islf_replica_desc *descs, int32_t n_reps, int32_t spin_format,
                                         int32_t tile, int32_t grid, int32_t *shapes, int32_t *items,
                                         int32_t items_cap, int32_t *n_items, int32_t *first, int32_t first_cap,
                                         int32_t *n_first)
{
    if (!descs || !n_items || !n_first) return fail(ISLF_EINVAL, "NULL argument");
    if (n_reps < 1) return fail(ISLF_EINVAL, "n_reps must be >= 1");
    if (spin_format != ISLF_SPIN_INT8 && spin_format != ISLF_SPIN_BITPACK)
        return fail(ISLF_EINVAL, "invalid spin format %d", spin_format);
    if (tile < -1 || tile >= num_tiles_of(spin_format)) return fail(ISLF_EINVAL, "invalid tile %d", tile);
    if (grid < 1 || grid > (1 << 20)) return fail(ISLF_EINVAL, "invalid workgroup count %d", grid);
    if (items_cap < 0 || first_cap < 0) return fail(ISLF_EINVAL, "negative capacity");
    std::vector<Entry> S, M;
    for (int r = 0; r < n_reps; ++r) {
        islf_status st = validate(descs + r);
        if (st != ISLF_OK) return st;
        Replica R;
        R.desc = descs[r];
        R.tile = tile >= 0 ? tile : default_tile(descs + r, spin_format);
        build_work(R, r, spin_format);
        if (shapes) {
            shapes[4 * r + 0] = R.tile;
            shapes[4 * r + 1] = R.d.i8_tj;
            shapes[4 * r + 2] = R.d.i8_ty;
            shapes[4 * r + 3] = R.d.i8_mx;
        }
        S.insert(S.end(), R.slab.begin(), R.slab.end());
        M.insert(M.end(), R.main.begin(), R.main.end());
    }
    std::vector<Entry> it;
    std::vector<int> fi;
    partition_items(S, M, grid, it, fi, tail_taper(spin_format));
    *n_items = (int32_t)it.size();
    *n_first = (int32_t)fi.size();
    if ((items && (int64_t)it.size() > items_cap) || (first && (int64_t)fi.size() > first_cap))
        return fail(ISLF_ERANGE, "plan needs %zu items and %zu offsets", it.size(), fi.size());
    if (items)
        for (size_t i = 0; i < it.size(); ++i) {
            const Entry &e = it[i];
            const int32_t v[6] = {e.rep, e.x0, e.y0, e.j0, e.nsteps, e.kind};
            for (int k = 0; k < 6; ++k) items[6 * i + k] = v[k];
        }
    if (first)
        for (size_t i = 0; i < fi.size(); ++i) first[i] = fi[i];
    return ISLF_OK;
}

extern "C" islf_status islf_batch_add(islf_ctx *ctx, const islf_replica_desc *desc, int32_t *slot)
{
    if (!ctx || !slot) return fail(ISLF_EINVAL, "NULL argument");
    int s = -1;
    islf_status st = add_replica(ctx, desc, &s);
    if (st != ISLF_OK) return st;
    *slot = s;
    return sync_tables(ctx);
}

extern "C" islf_status islf_batch_retire(islf_ctx *ctx, int32_t slot)
{
    islf_status st = check_rep(ctx, slot);
    if (st != ISLF_OK) return st;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    Replica &R = ctx->reps[slot];
    R.live = false;
    R.t_host = 0;
    R.failed = false;
    // the slot's memory goes back to the allocator, so the device memory a
    // context holds follows its live replicas
    dev_free(ctx, R.mem);
    R.mem = nullptr;
    R.mem_bytes = 0;
    R.main.clear();
    R.slab.clear();
    ctx->dirty = true;
    return sync_tables(ctx);
}

extern "C" islf_status islf_graph_capture(islf_ctx *ctx, uint32_t k_sweeps)
{
    if (!ctx) return fail(ISLF_EINVAL, "NULL context");
    if (k_sweeps < 1) return fail(ISLF_EINVAL, "k_sweeps must be >= 1");
    if (!ctx->stream) return fail(ISLF_ESTATE, "graph capture needs a non-default stream");
    islf_status st = check_none_failed(ctx);
    if (st != ISLF_OK) return st;
    st = prepare_plans(ctx, ctx->exec);
    if (st != ISLF_OK) return st;
    destroy_graphs(ctx);
    // concurrent groups: one graph per group, captured on the group's own
    // stream, so that replays run each group on a stream the context owns
    // (the streams a runtime picks for the branches of one multi-stream graph
    // may share a hardware queue and serialise the groups)
    const bool grouped = ctx->exec == ISLF_EXEC_BATCHED && num_groups(ctx) > 1;
    const int G = grouped ? num_groups(ctx) : 1;
    for (int gi = 0; gi < G; ++gi) {
        hipStream_t sg = group_stream(ctx, gi, G);
        HIP_TRY(hipStreamBeginCapture(sg, hipStreamCaptureModeThreadLocal));
        hipError_t ee = hipSuccess;
        if (grouped) ee = enqueue_group(ctx, gi, k_sweeps);
        else st = enqueue_sweeps(ctx, k_sweeps);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(sg, &g);
        if (st != ISLF_OK || ee != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            destroy_graphs(ctx);
            return st != ISLF_OK ? st : fail(ISLF_EDEVICE, "launch during capture failed: %s", hipGetErrorString(ee));
        }
        if (e != hipSuccess) {
            destroy_graphs(ctx);
            return fail(ISLF_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        }
        ctx->graphs.push_back(g);
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            destroy_graphs(ctx);
            return fail(ISLF_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
        }
        ctx->graph_execs.push_back(ex);
    }
    ctx->graph_sweeps = k_sweeps;
    ctx->graph_valid = true;
    return ISLF_OK;
}

extern "C" islf_status islf_run_graph(islf_ctx *ctx, uint32_t n_replays)
{
    if (!ctx) return fail(ISLF_EINVAL, "NULL context");
    if (!ctx->graph_valid || ctx->dirty) return fail(ISLF_ESTATE, "no valid captured graph");
    islf_status st = check_none_failed(ctx);
    if (st != ISLF_OK) return st;
    st = check_sweep_range(ctx, (uint64_t)ctx->graph_sweeps * n_replays);
    if (st != ISLF_OK) return st;
    const int G = (int)ctx->graph_execs.size();
    if (G > 1) HIP_TRY(fork_groups(ctx, G));
    for (uint32_t i = 0; i < n_replays; ++i)
        for (int g = 0; g < G; ++g) HIP_TRY(hipGraphLaunch(ctx->graph_execs[g], group_stream(ctx, g, G)));
    if (G > 1) HIP_TRY(join_groups(ctx, G));
    for (int r : ctx->live) ctx->reps[r].t_host += (uint64_t)ctx->graph_sweeps * n_replays;
    return ISLF_OK;
}

extern "C" islf_status islf_num_tiles(int32_t spin_format, int32_t *n)
{
    if (!n) return fail(ISLF_EINVAL, "NULL output");
    if (spin_format != ISLF_SPIN_INT8 && spin_format != ISLF_SPIN_BITPACK)
        return fail(ISLF_EINVAL, "invalid spin format %d", spin_format);
    *n = num_tiles_of(spin_format);
    return ISLF_OK;
}

extern "C" islf_status islf_get_tile(const islf_ctx *ctx, int32_t rep, int32_t *tile)
{
    islf_status st = check_rep(ctx, rep);
    if (st != ISLF_OK) return st;
    if (!tile) return fail(ISLF_EINVAL, "NULL output");
    *tile = ctx->reps[rep].tile;
    return ISLF_OK;
}

extern "C" islf_status islf_set_tile(islf_ctx *ctx, int32_t rep, int32_t tile)
{
    islf_status st = check_rep(ctx, rep);
    if (st != ISLF_OK) return st;
    if (tile < 0 || tile >= num_tiles_of(ctx->fmt)) return fail(ISLF_EINVAL, "tile %d out of range", tile);
    Replica &R = ctx->reps[rep];
    R.tile = tile;
    build_work(R, rep, ctx->fmt);
    ctx->dirty = true;
    return ISLF_OK;
}

// Timed runs per autotune trial (the shortest counts), and per finalist of
// the launch-configuration search.
constexpr int kTrialRuns = 3;
constexpr int kFinalRuns = 6;
constexpr int kFinalists = 4;

// Times one tile variant for one size class: the class's replicas sweep
// `sweeps` times in the batched form over a plan of their own (events on the
// context stream).  Spins, records and state are restored afterwards by the
// caller.
static islf_status time_variant(islf_ctx *c, const std::vector<int> &cls, int tile, uint32_t sweeps, double *ms)
{
    std::vector<Entry> M, S;
    for (int r : cls) {
        Replica &R = c->reps[r];
        R.tile = tile;
        build_work(R, r, c->fmt);
        M.insert(M.end(), R.main.begin(), R.main.end());
        S.insert(S.end(), R.slab.begin(), R.slab.end());
        HIP_TRY(hipMemcpyAsync(c->d_desc + r, &R.d, sizeof(RepDesc), hipMemcpyHostToDevice, c->stream));
    }
    Plan plan;
    islf_status st = build_plan(c, plan, S, M, c->grid_override ? c->grid_override : c->sweep_slots);
    if (st != ISLF_OK) {
        free_plan(c, plan);
        return st;
    }
    int *dl = (int *)dev_alloc(c, sizeof(int) * cls.size());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = dl ? hipSuccess : hipErrorOutOfMemory;
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    if (err == hipSuccess) err = hipMemcpyAsync(dl, cls.data(), sizeof(int) * cls.size(), hipMemcpyHostToDevice, c->stream);
    // one warm-up sweep, then the shortest of three timed runs (a single run
    // of a few sweeps is too noisy to rank variants)
    if (err == hipSuccess) err = enqueue_plan(c, plan, dl, (int)cls.size(), 1);
    float t = 0.f;
    for (int run = 0; run < kTrialRuns && err == hipSuccess; ++run) {
        err = hipEventRecord(e0, c->stream);
        if (err == hipSuccess) err = enqueue_plan(c, plan, dl, (int)cls.size(), sweeps);
        if (err == hipSuccess) err = hipEventRecord(e1, c->stream);
        if (err == hipSuccess) err = hipStreamSynchronize(c->stream);
        float tr = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&tr, e0, e1);
        if (err == hipSuccess && (run == 0 || tr < t)) t = tr;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    free_plan(c, plan);
    dev_free(c, dl);
    if (err != hipSuccess) return fail(ISLF_EDEVICE, "autotune trial failed: %s", hipGetErrorString(err));
    *ms = t;
    return ISLF_OK;
}

extern "C" islf_status islf_autotune(islf_ctx *ctx, uint32_t sweeps)
{
    if (!ctx) return fail(ISLF_EINVAL, "NULL context");
    if (sweeps < 1) return fail(ISLF_EINVAL, "sweeps must be >= 1");
    islf_status st = sync_tables(ctx);
    if (st != ISLF_OK) return st;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    // size classes: replicas of one shape share a variant
    std::vector<std::vector<int>> classes;
    for (int r : ctx->live) {
        bool placed = false;
        for (auto &cl : classes) {
            const islf_replica_desc &a = ctx->reps[cl[0]].desc, &b = ctx->reps[r].desc;
            if (a.Lx == b.Lx && a.Ly == b.Ly && a.Lz == b.Lz) {
                cl.push_back(r);
                placed = true;
                break;
            }
        }
        if (!placed) classes.push_back({r});
    }
    // back up every live replica's memory block and state
    std::vector<void *> backup(ctx->reps.size(), nullptr);
    RepState *st_backup = (RepState *)dev_alloc(ctx, sizeof(RepState) * ctx->slot_capacity);
    islf_status result = st_backup ? ISLF_OK : fail(ISLF_ENOMEM, "cannot back up replica state");
    for (int r : ctx->live) {
        if (result != ISLF_OK) break;
        Replica &R = ctx->reps[r];
        backup[r] = dev_alloc(ctx, R.mem_bytes);
        if (!backup[r]) result = fail(ISLF_ENOMEM, "cannot back up replica %d", r);
        else if (hipMemcpyAsync(backup[r], R.mem, R.mem_bytes, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess)
            result = fail(ISLF_EDEVICE, "backup copy failed");
    }
    if (result == ISLF_OK &&
        hipMemcpyAsync(st_backup, ctx->d_state, sizeof(RepState) * ctx->slot_capacity, hipMemcpyDeviceToDevice,
                       ctx->stream) != hipSuccess)
        result = fail(ISLF_EDEVICE, "state backup failed");
    auto restore = [&]() -> islf_status {
        for (int r : ctx->live)
            HIP_TRY(hipMemcpyAsync(ctx->reps[r].mem, backup[r], ctx->reps[r].mem_bytes, hipMemcpyDeviceToDevice,
                                   ctx->stream));
        HIP_TRY(hipMemcpyAsync(ctx->d_state, st_backup, sizeof(RepState) * ctx->slot_capacity,
                               hipMemcpyDeviceToDevice, ctx->stream));
        return ISLF_OK;
    };
    for (auto &cl : classes) {
        if (result != ISLF_OK) break;
        const int orig = ctx->reps[cl[0]].tile;
        // the fastest variant, if it beats the replica's own by 1%
        double best = 1e300, orig_ms = 1e300;
        int best_tile = orig;
        for (int tile = 0; tile < num_tiles_of(ctx->fmt) && result == ISLF_OK; ++tile) {
            double ms = 0;
            result = time_variant(ctx, cl, tile, sweeps, &ms);
            if (result == ISLF_OK) result = restore();
            if (result == ISLF_OK && tile == orig) orig_ms = ms;
            if (result == ISLF_OK && ms < best) {
                best = ms;
                best_tile = tile;
            }
        }
        if (best_tile != orig && orig_ms < 1e300 && best >= 0.99 * orig_ms) best_tile = orig;
        for (int r : cl) {
            ctx->reps[r].tile = (result == ISLF_OK) ? best_tile : orig;
            build_work(ctx->reps[r], r, ctx->fmt);
        }
    }
    if (result == ISLF_OK) {
        islf_status rs = restore();
        if (rs != ISLF_OK) result = rs;
    }
    // the launch configuration of the context's form on the whole batch:
    // batched: concurrent groups x workgroups per launch x share taper;
    // persistent: barrier form x grid (up to the co-residency bound) x taper.
    // Each trial captures `sweeps` sweeps as graphs and times replays of
    // them; the chains advance during the trials and are restored once
    // afterwards.
    if (result == ISLF_OK && !ctx->live.empty() &&
        (ctx->exec == ISLF_EXEC_BATCHED || ctx->exec == ISLF_EXEC_PERSISTENT)) {
        ctx->dirty = true;
        result = sync_tables(ctx);
        const int keep_groups = ctx->groups_req, keep_grid = ctx->grid_override;
        const double keep_taper = ctx->taper_override;
        struct Trial { int groups, grid; double taper; int team; };
        const int keep_team = ctx->team_mode;
        std::vector<Trial> trials;
        const double tapers[] = {0.0, 0.1, 0.2};
        if (ctx->exec == ISLF_EXEC_BATCHED) {
            const int nl = (int)ctx->live.size();
            for (int G = 1; G <= std::min(4, nl); ++G) {
                const int base = G == 1 ? ctx->sweep_slots : std::max(64, (3 * ctx->resident_slots + G) / (2 * G));
                for (double f : {0.5, 1.0, 1.5})
                    for (double tp : tapers) trials.push_back(Trial{G, std::max(32, (int)(base * f + 0.5)), tp, keep_team});
            }
        } else {
            // up to one workgroup per CU below the bound, like the default grid
            const int per_cu = std::max(1, ctx->persistent_bound / std::max(1, ctx->num_cu));
            const int top = std::max(1, per_cu - 1);
            // the persistent shares step down by dispatch round: stronger tapers
            for (int team = 0; team <= 1; ++team)
                for (int k = std::max(1, top - 2); k <= top; ++k)
                    for (double tp : {0.0, 0.2, 0.4, 0.6})
                        trials.push_back(Trial{0, std::min(ctx->num_cu * k, ctx->persistent_bound), tp, team});
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (result == ISLF_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
            result = fail(ISLF_EDEVICE, "cannot create events");
        // one trial: the shortest of `runs` timed replays of a captured graph
        // of `sweeps` sweeps after one untimed replay (eager launches without
        // a stream to capture on)
        auto time_trial = [&](const Trial &t, int runs, float *best_ms) -> islf_status {
            ctx->groups_req = t.groups ? t.groups : keep_groups;
            ctx->grid_override = t.grid;
            ctx->taper_override = t.taper;
            ctx->team_mode = t.team;
            ctx->groups_valid = false;
            ctx->batched.valid = false;
            ctx->persistent.valid = false;
            islf_status rs = prepare_plans(ctx, ctx->exec);
            if (rs != ISLF_OK) return rs;
            hipError_t e = hipSuccess;
            int G = 1;
            if (ctx->stream) {
                rs = islf_graph_capture(ctx, sweeps);
                if (rs != ISLF_OK) return rs;
                G = (int)ctx->graph_execs.size();
            }
            for (int run = 0; run <= runs && e == hipSuccess; ++run) {
                if (run == 1) e = hipEventRecord(e0, ctx->stream);
                if (e == hipSuccess && ctx->stream) {
                    if (G > 1) e = fork_groups(ctx, G);
                    for (int g = 0; g < G && e == hipSuccess; ++g)
                        e = hipGraphLaunch(ctx->graph_execs[g], group_stream(ctx, g, G));
                    if (e == hipSuccess && G > 1) e = join_groups(ctx, G);
                } else if (e == hipSuccess) {
                    rs = enqueue_sweeps(ctx, run == 0 ? 1 : sweeps);
                    if (rs != ISLF_OK) break;
                }
                if (run >= 1 && e == hipSuccess) {
                    e = hipEventRecord(e1, ctx->stream);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    float ms = 0.f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                    if (e == hipSuccess && (run == 1 || ms < *best_ms)) *best_ms = ms;
                    if (e == hipSuccess && run < runs) e = hipEventRecord(e0, ctx->stream);
                }
            }
            if (ctx->stream) destroy_graphs(ctx);
            if (rs != ISLF_OK) return rs;
            if (e != hipSuccess) return fail(ISLF_EDEVICE, "autotune trial failed: %s", hipGetErrorString(e));
            return ISLF_OK;
        };
        // first pass over every trial, then the fastest few and the entry
        // configuration again with more runs; the entry configuration stays
        // unless a finalist beats it by 1%
        const Trial entry{keep_groups, keep_grid, keep_taper, keep_team};
        std::vector<std::pair<float, size_t>> first;
        for (size_t i = 0; i < trials.size() && result == ISLF_OK; ++i) {
            float ms = 0.f;
            result = time_trial(trials[i], kTrialRuns, &ms);
            if (result == ISLF_OK) first.push_back({ms, i});
        }
        Trial best_t = entry;
        if (result == ISLF_OK) {
            std::sort(first.begin(), first.end());
            float entry_ms = 0.f;
            result = time_trial(entry, kFinalRuns, &entry_ms);
            float best = entry_ms;
            for (size_t k = 0; k < first.size() && (int)k < kFinalists && result == ISLF_OK; ++k) {
                float ms = 0.f;
                result = time_trial(trials[first[k].second], kFinalRuns, &ms);
                if (result == ISLF_OK && ms < best && ms < 0.99f * entry_ms) {
                    best = ms;
                    best_t = trials[first[k].second];
                }
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        ctx->groups_req = (result == ISLF_OK && best_t.groups) ? best_t.groups : keep_groups;
        ctx->grid_override = result == ISLF_OK ? best_t.grid : keep_grid;
        ctx->taper_override = result == ISLF_OK ? best_t.taper : keep_taper;
        ctx->team_mode = result == ISLF_OK ? best_t.team : keep_team;
        ctx->groups_valid = false;
        ctx->batched.valid = false;
        ctx->persistent.valid = false;
        ctx->graph_valid = false;
        if (result == ISLF_OK) {
            islf_status rs = restore();
            if (rs != ISLF_OK) result = rs;
        }
    }
    if (hipStreamSynchronize(ctx->stream) != hipSuccess && result == ISLF_OK)
        result = fail(ISLF_EDEVICE, "autotune synchronisation failed");
    for (void *b : backup) dev_free(ctx, b);
    dev_free(ctx, st_backup);
    ctx->dirty = true;
    if (result != ISLF_OK) return result;
    return sync_tables(ctx);
}

// 32-bit words per (x, y) row of the spin array
static long profile_row_words(const Replica &R)
{
    return R.d.fmt == ISLF_SPIN_INT8 ? R.d.RB / 4 : 2l * R.d.Wq;
}

extern "C" islf_status islf_layer_profile(islf_ctx *ctx, int32_t rep, int32_t *dev_out)
{
    islf_status st = check_rep(ctx, rep);
    if (st != ISLF_OK) return st;
    if (!dev_out) return fail(ISLF_EINVAL, "NULL output");
    if (ctx->reps[rep].failed)
        return fail(ISLF_ESTATE, "replica %d was cut short by a failed persistent launch", rep);
    st = sync_tables(ctx);
    if (st != ISLF_OK) return st;
    const Replica &R = ctx->reps[rep];
    HIP_TRY(launch_layer_profile(ctx->d_desc, rep, (long)R.desc.Lx * R.desc.Ly, profile_row_words(R), dev_out,
                                 nullptr, ctx->stream));
    return ISLF_OK;
}

extern "C" islf_status islf_layer_profile_add(islf_ctx *ctx, int32_t rep, int64_t *dev_acc)
{
    islf_status st = check_rep(ctx, rep);
    if (st != ISLF_OK) return st;
    if (!dev_acc) return fail(ISLF_EINVAL, "NULL accumulator");
    if (ctx->reps[rep].failed)
        return fail(ISLF_ESTATE, "replica %d was cut short by a failed persistent launch", rep);
    st = sync_tables(ctx);
    if (st != ISLF_OK) return st;
    const Replica &R = ctx->reps[rep];
    HIP_TRY(launch_layer_profile(ctx->d_desc, rep, (long)R.desc.Lx * R.desc.Ly, profile_row_words(R), nullptr,
                                 (long long *)dev_acc, ctx->stream));
    return ISLF_OK;
}

extern "C" islf_status islf_set_grid(islf_ctx *ctx, int32_t workgroups)
{
    if (!ctx) return fail(ISLF_EINVAL, "NULL context");
    if (workgroups < 0 || workgroups > (1 << 20)) return fail(ISLF_EINVAL, "invalid workgroup count %d", workgroups);
    if (ctx->exec == ISLF_EXEC_PERSISTENT && workgroups > ctx->persistent_bound)
        return fail(ISLF_ERANGE, "persistent grid %d exceeds the co-residency bound %d of this device", workgroups,
                    ctx->persistent_bound);
    ctx->grid_override = workgroups;
    ctx->batched.valid = false;
    ctx->persistent.valid = false;
    ctx->groups_valid = false;
    for (Plan &p : ctx->plain) p.valid = false;
    ctx->graph_valid = false;
    return ISLF_OK;
}

extern "C" islf_status islf_set_groups(islf_ctx *ctx, int32_t groups)
{
    if (!ctx) return fail(ISLF_EINVAL, "NULL context");
    if (groups < 0 || groups > kMaxStreamGroups) return fail(ISLF_EINVAL, "invalid group count %d", groups);
    ctx->groups_req = groups;
    ctx->groups_valid = false;
    ctx->graph_valid = false;
    return ISLF_OK;
}

extern "C" islf_status islf_get_groups(const islf_ctx *ctx, int32_t *groups)
{
    if (!ctx || !groups) return fail(ISLF_EINVAL, "NULL argument");
    *groups = num_groups(ctx);
    return ISLF_OK;
}

extern "C" islf_status islf_get_grid(const islf_ctx *ctx, int32_t *workgroups)
{
    if (!ctx || !workgroups) return fail(ISLF_EINVAL, "NULL argument");
    if (ctx->exec == ISLF_EXEC_PERSISTENT)
        *workgroups = ctx->grid_override ? ctx->grid_override : ctx->persistent_grid;
    else
        *workgroups = launch_grid(ctx, ctx->exec);
    return ISLF_OK;
}

extern "C" islf_status islf_phase_timings(islf_ctx *ctx, uint32_t n_sweeps, double *mean_ms, uint32_t *launches)
{
    if (!ctx || !mean_ms || !launches) return fail(ISLF_EINVAL, "NULL argument");
    if (n_sweeps < 1) return fail(ISLF_EINVAL, "n_sweeps must be >= 1");
    islf_status st = sync_tables(ctx);
    if (st == ISLF_OK && !ctx->batched.valid && !ctx->live.empty()) {
        std::vector<Entry> S, M;
        for (int r : ctx->live) {
            S.insert(S.end(), ctx->reps[r].slab.begin(), ctx->reps[r].slab.end());
            M.insert(M.end(), ctx->reps[r].main.begin(), ctx->reps[r].main.end());
        }
        st = build_plan(ctx, ctx->batched, S, M, ctx->grid_override ? ctx->grid_override : ctx->sweep_slots);
    }
    if (st != ISLF_OK) return st;
    st = check_sweep_range(ctx, n_sweeps);
    if (st != ISLF_OK) return st;
    const int nl = (int)ctx->live.size();
    std::vector<hipEvent_t> ev(4 * (size_t)n_sweeps + 2, nullptr);
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &f : ev)
                if (f) (void)hipEventDestroy(f);
            return fail(ISLF_EDEVICE, "cannot create events");
        }
    hipError_t err = nl ? enqueue_plan(ctx, ctx->batched, ctx->d_live, nl, n_sweeps, ev.data()) : hipSuccess;
    if (err == hipSuccess) err = hipStreamSynchronize(ctx->stream);
    double sum[3] = {0, 0, 0};
    uint32_t cnt[3] = {0, 0, 0};
    if (err == hipSuccess && nl) {
        for (size_t k = 0; k <= 2 * (size_t)n_sweeps; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]) != hipSuccess) continue;
            const int kind = k == 2 * (size_t)n_sweeps ? 2 : (int)(k & 1);
            sum[kind] += ms;
            cnt[kind] += 1;
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (err != hipSuccess) return fail(ISLF_EDEVICE, "timed sweeps failed: %s", hipGetErrorString(err));
    for (int r : ctx->live) ctx->reps[r].t_host += n_sweeps;
    for (int k = 0; k < 3; ++k) {
        mean_ms[k] = cnt[k] ? sum[k] / cnt[k] : 0.0;
        launches[k] = cnt[k];
    }
    return ISLF_OK;
}

extern "C" islf_status islf_replica_means(islf_ctx *ctx, int32_t rep, uint64_t first, uint32_t count, double *out)
{
    islf_status st = check_rep(ctx, rep);
    if (st != ISLF_OK) return st;
    if (!out) return fail(ISLF_EINVAL, "NULL output");
    st = check_records(ctx, rep, first, count);
    if (st != ISLF_OK) return st;
    st = check_intact(ctx, rep);
    if (st != ISLF_OK) return st;
    int *dl = (int *)dev_alloc(ctx, sizeof(int));
    double *tmp = (double *)dev_alloc(ctx, sizeof(double) * 5);
    hipError_t e = (dl && tmp) ? hipSuccess : hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipMemcpyAsync(dl, &rep, sizeof(int), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = launch_means(ctx->d_desc, dl, 1, first, count, tmp, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, sizeof(double) * 5, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    dev_free(ctx, dl);
    dev_free(ctx, tmp);
    if (e != hipSuccess) return fail(ISLF_EDEVICE, "replica means failed: %s", hipGetErrorString(e));
    return ISLF_OK;
}

extern "C" islf_status islf_device_bytes(const islf_ctx *ctx, uint64_t *total, uint64_t *replica_bytes)
{
    if (!ctx || !total) return fail(ISLF_EINVAL, "NULL argument");
    *total = (uint64_t)ctx->dev_bytes;
    if (replica_bytes) {
        uint64_t r = 0;
        for (const Replica &R : ctx->reps)
            if (R.mem) r += R.mem_bytes;
        *replica_bytes = r;
    }
    return ISLF_OK;
}

// Test support, not part of the public header: raises the persistent
// kernel's error word from the host, as a block that gave up at a grid
// barrier would, so that the failure path can be exercised without a launch
// that really fails.  Every block of the next persistent launch then stops
// at its first barrier.
extern "C" islf_status islf_testing_raise_barrier_error(islf_ctx *ctx)
{
    if (!ctx) return fail(ISLF_EINVAL, "NULL context");
    const unsigned long long one = 1;
    HIP_TRY(hipMemcpyAsync(&ctx->d_sync->error.v, &one, sizeof one, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return ISLF_OK;
}

extern "C" islf_status islf_set_taper(islf_ctx *ctx, double taper)
{
    if (!ctx) return fail(ISLF_EINVAL, "NULL context");
    if (!(taper < 1.0)) return fail(ISLF_EINVAL, "taper must be below 1 (got %g)", taper);
    ctx->taper_override = taper < 0.0 ? -1.0 : taper;
    ctx->batched.valid = false;
    ctx->persistent.valid = false;
    ctx->groups_valid = false;
    ctx->graph_valid = false;
    return ISLF_OK;
}

extern "C" islf_status islf_get_taper(const islf_ctx *ctx, double *taper)
{
    if (!ctx || !taper) return fail(ISLF_EINVAL, "NULL argument");
    if (ctx->taper_override >= 0.0) *taper = ctx->taper_override;
    else if (ctx->exec == ISLF_EXEC_PERSISTENT)
        *taper = kPersistentTaper;
    else *taper = tail_taper(ctx->fmt);
    return ISLF_OK;
}

extern "C" islf_status islf_set_barriers(islf_ctx *ctx, int32_t mode)
{
    if (!ctx) return fail(ISLF_EINVAL, "NULL context");
    if (mode != ISLF_BARRIER_GRID && mode != ISLF_BARRIER_TEAM && mode != ISLF_BARRIER_AUTO)
        return fail(ISLF_EINVAL, "invalid barrier mode %d", mode);
    ctx->team_mode = mode == ISLF_BARRIER_TEAM ? 1 : mode == ISLF_BARRIER_GRID ? 0 : -1;
    ctx->persistent.valid = false;
    ctx->graph_valid = false;
    return ISLF_OK;
}

extern "C" islf_status islf_get_barriers(const islf_ctx *ctx, int32_t *mode)
{
    if (!ctx || !mode) return fail(ISLF_EINVAL, "NULL argument");
    // the form the next persistent launch uses
    const int grid = ctx->grid_override ? ctx->grid_override : ctx->persistent_grid;
    *mode = use_teams(ctx, grid) ? ISLF_BARRIER_TEAM : ISLF_BARRIER_GRID;
    return ISLF_OK;
}
