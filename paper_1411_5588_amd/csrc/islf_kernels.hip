// gfx950 kernels of libislf: checkerboard Metropolis sweeps of the thin-film
// Ising model (arXiv:1411.5588, Sec. II.A Eq. 1 with the y boundaries of
// Eq. 11; Appendix: checkerboard update), fused observable reductions, random
// initial states, full-recompute observables, record bookkeeping, means and
// the field thermodynamic integration (Eq. 9 / Eq. 22).
//
// The path is integer stencil work plus Philox4x32-10: no matrix cores.  Two
// spin formats:
//  * int8: one byte per site, 1 = up, 0 = down; each row (x, y) is split
//    into its even-z sublattice (z = 2i at byte i) and its odd-z sublattice
//    (z = 2i+1 at byte Hp + i), Hp = 8*ceil(Lz/16), row index x*Ly + y,
//    padding bytes 0.  The sites of one phase in a row are one sublattice,
//    so a thread owns an 8-byte column of it: 8 sites of the phase, two
//    Philox calls, one 8-byte store of its own sites only; neighbour counts
//    of all 8 bytes are formed with word-wide adds (each byte holds 0/1, sums
//    stay below 8, so no carry crosses a byte).
//  * bit-packed: one bit per site, each row split into its even-z and odd-z
//    sublattices of Lz/2 bits.  A thread owns one 32-bit word of one
//    sublattice row (32 sites of the same phase, 8 Philox calls); neighbour
//    counts are bit-sliced with full adders.
// Both formats draw the same Philox word for the same site, so they give the
// same Markov chain.
#include <mutex>

#include "islf_internal.h"

#pragma clang fp contract(off)

namespace islf {

// a ^ b ^ c in one gfx950 three-input bitwise op (truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 multiplies
// whose halves are xored into the other counter words with the round key; the
// key advances by the Weyl constants after each round.
// ---------------------------------------------------------------------------
// The first round's product of c0 = base + OFF is formed as one multiply-add,
// M0 base + M0 OFF, which is M0 c0 whenever base + OFF < 2^32 (every counter
// of a valid site: the group index is checked against 2^32 when a replica is
// created); OFF = 0 is the plain generator.
template <uint32_t OFF = 0>
__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1, uint32_t out[4])
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)0xD2511F53u * c0 + (r == 0 ? (uint64_t)0xD2511F53u * OFF : 0ull);
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(pb >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(pa >> 32), c3, k1);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

constexpr uint64_t kOnes8 = 0x0101010101010101ull;

__device__ __forceinline__ uint32_t bytesum64(uint64_t v)
{
    return __builtin_amdgcn_sad_u8((uint32_t)v, 0u, __builtin_amdgcn_sad_u8((uint32_t)(v >> 32), 0u, 0u));
}

struct Acc {
    int dB, dM, dM1, dMn;
};

// Wave64 + workgroup reduction of the four partial sums, then one atomic add
// per quantity into the replica's spread accumulator of the current sweep.
__device__ void flush_acc(Acc &a, long long *acc_base, uint32_t t, int slot)
{
    __shared__ int red[4][kBlock / 64];
    int v[4] = {a.dB, a.dM, a.dM1, a.dMn};
    // every lane of the workgroup reaches this point: full-wave DPP sums
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = __reduce_add_sync(~0ull, v[k]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) red[k][wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        int s = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) s += red[threadIdx.x][w];
        if (s != 0) {
            long long *dst = acc_base + ((size_t)(t & 1) * kAccSlots + slot) * 4 + threadIdx.x;
            atomicAdd((unsigned long long *)dst, (unsigned long long)(long long)s);
        }
    }
    __syncthreads();
    a.dB = a.dM = a.dM1 = a.dMn = 0;
}

// Per-replica lookup tables staged in LDS: 64-bit thresholds (used by the
// seam and bit-packed paths and by replicas with never-accepted moves),
// thr - 1 as 32 bits and the packed (dB, dM) change of a flip.
struct TD {
    uint32_t thr_m1;
    int32_t dpack;
};
struct Tables {
    uint64_t thr[kThrEntries];
    TD td[kThrEntries];
    // bulk class, two neighbouring sites at once (bit-packed main tiles):
    // entry k, the index bits of the two sites interleaved (even bits: the
    // first site's e = 8u + cnt, odd bits: the second's), holds their thr - 1
    uint2 pair[256];
};

template <bool PAIRS = false>
__device__ __forceinline__ void load_tables(const RepDesc &d, Tables *t)
{
    for (int k = threadIdx.x; k < kThrEntries; k += blockDim.x) {
        t->thr[k] = d.thr[k];
        t->td[k].thr_m1 = d.thr_m1[k];
        t->td[k].dpack = d.dpack[k];
    }
    if (PAIRS)
        for (int k = threadIdx.x; k < 256; k += blockDim.x) {
            const int ev = (k & 1) | ((k >> 1) & 2) | ((k >> 2) & 4) | ((k >> 3) & 8);
            const int od = ((k >> 1) & 1) | ((k >> 2) & 2) | ((k >> 3) & 4) | ((k >> 4) & 8);
            t->pair[k] = make_uint2(d.thr_m1[ev], d.thr_m1[od]);
        }
}

// Per-replica parameters as the update loop uses them: loaded once per
// replica change from the descriptor table, uniform across the workgroup (the
// compiler keeps them in scalar registers).
struct RepView {
    uint8_t *spins;
    long long *acc;
    int Lx, Ly, Lz, C, Wq, K;
    uint32_t Hp, RB;        // int8 sublattice row and row bytes
    int seam_reflect, seam_invert;
    uint32_t key0, key1, replica, t;
    int tj, ty, mx;          // marching tile (tj = 0: linear tiles)
    int my_ty, my_tj;        // this thread's row and column inside a box tile
    bool never;              // some move can never be accepted (thr == 0)
};

__device__ __forceinline__ RepView load_view(const RepDesc *__restrict__ descs, const RepState *__restrict__ st,
                                             int rep, uint32_t t_offset)
{
    const RepDesc &d = descs[rep];
    RepView v;
    v.spins = d.spins;
    v.acc = d.acc;
    v.Lx = d.Lx; v.Ly = d.Ly; v.Lz = d.Lz; v.C = d.C; v.Wq = d.Wq; v.K = d.K;
    v.Hp = (uint32_t)d.Hp;
    v.RB = (uint32_t)d.RB;
    v.seam_reflect = d.seam_reflect;
    v.seam_invert = d.seam_invert;
    v.key0 = d.key0; v.key1 = d.key1; v.replica = d.replica;
    v.t = st[rep].t + t_offset;
    v.tj = d.i8_tj;
    v.ty = d.i8_ty;
    v.mx = d.i8_mx;
    v.my_ty = v.tj > 0 ? (int)threadIdx.x / v.tj : 0;
    v.my_tj = (int)threadIdx.x - v.my_ty * v.tj;
    v.never = d.never_mask != 0;
    return v;
}

// ---------------------------------------------------------------------------
// int8 format: update the current-phase sites of one 8-byte column.
// Byte offsets are 32-bit (a replica's spin array is below 4 GiB).
// ---------------------------------------------------------------------------
// Loads through the global address space (the spin arrays always live in
// device memory), addressed as a uniform base plus a 32-bit offset.
typedef __attribute__((address_space(1))) const uint8_t gcu8;
typedef __attribute__((address_space(1))) const uint32_t gcu32;
typedef __attribute__((address_space(1))) const uint64_t gcu64;
typedef __attribute__((address_space(1))) uint64_t gu64;
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) uint8_t gu8;

// Lattice accesses.  COH (the persistent kernel) makes them relaxed
// device-scope atomics, which the compiler marks device-coherent: stores
// write through the XCD's L2 and loads do not use a stale copy in it, so a
// block on any XCD sees another's stores once they are complete, and the
// grid barrier needs no L2 write-back or invalidate (see grid_barrier).
template <bool COH>
__device__ __forceinline__ uint64_t ld64(const uint8_t *base, uint32_t off)
{
    gu64 *p = (gu64 *)((gcu8 *)base + off);
    if (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
}
template <bool COH>
__device__ __forceinline__ uint32_t ld32(const uint8_t *base, uint32_t off)
{
    gu32 *p = (gu32 *)((gcu8 *)base + off);
    if (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
}
template <bool COH>
__device__ __forceinline__ uint64_t ld8(const uint8_t *base, uint32_t off)
{
    gu8 *p = (gu8 *)((gcu8 *)base + off);
    if (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
}
template <bool COH>
__device__ __forceinline__ void st64(uint8_t *base, uint32_t off, uint64_t v)
{
    gu64 *p = (gu64 *)((gcu8 *)base + off);
    if (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}
template <bool COH>
__device__ __forceinline__ void st32(uint8_t *base, uint32_t off, uint32_t v)
{
    gu32 *p = (gu32 *)((gcu8 *)base + off);
    if (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

// Bytes [0, nv) of an 8-byte column set.
__device__ __forceinline__ uint64_t byte_mask(int nv)
{
    return nv >= 8 ? ~0ull : ((1ull << (8 * nv)) - 1ull);
}

// One 8-byte column k of the phase's sublattice of row (x, y): 8 sites
// z = 2i + q, i = 8k .. 8k+7 (the last column of a row may hold fewer).
// Philox call c (counter g + 2c) draws for sites i = 8k + 4c .. 8k + 4c + 3
// (their 8-site group is i >> 2 = 2k + c, word i & 3).  Used by the
// seam-slab stages: any row, the y seam, 64-bit thresholds of any class.
template <bool COH>
__device__ __forceinline__ void i8_update_col(const RepView &v, int x, int y, int k, int parity,
                                              const uint64_t *sthr, Acc &a)
{
    const int Lx = v.Lx, Ly = v.Ly, K = v.K;
    const int Lzh = v.Lz >> 1;
    const uint32_t RB = v.RB, Hp = v.Hp;
    uint8_t *sp = v.spins;
    const int q = (parity + x + y) & 1;
    const uint32_t row = (uint32_t)x * (uint32_t)Ly + (uint32_t)y;
    const uint32_t rowoff = row * RB;
    const uint32_t co = 8u * (uint32_t)k;
    const uint32_t qo = (uint32_t)q * Hp + co;            // column offset inside a row
    const uint32_t own = rowoff + qo;
    const uint32_t oth = rowoff + (uint32_t)(q ^ 1) * Hp + co;
    const bool last = (k == K - 1);
    const int nv = last ? Lzh - 8 * (K - 1) : 8;

    // z neighbours from the other sublattice O of the row: q = 0 (z = 2i):
    // z+1 is odd index i, z-1 odd index i-1; q = 1 (z = 2i+1): z-1 is even
    // index i, z+1 even index i+1 (wrapping at the row's ends)
    const uint64_t O = ld64<COH>(sp, oth);
    uint64_t Z;
    if (q == 0) {
        const uint32_t eo = k > 0 ? oth - 1u : rowoff + Hp + (uint32_t)(Lzh - 1);
        Z = (O << 8) | ld8<COH>(sp, eo);
    } else {
        const uint32_t eo = last ? rowoff : oth + 8u;
        Z = (O >> 8) | (ld8<COH>(sp, eo) << (8 * (nv - 1)));
    }
    // y neighbours (the seam remaps x and inverts when eps = -1; a padding
    // byte may turn to 1 there, it is never a site) and x neighbours (a free
    // surface contributes 0)
    const uint32_t xs = v.seam_reflect ? (uint32_t)(Lx - 1 - x) : (uint32_t)x;
    const uint64_t seam_mask = v.seam_invert ? kOnes8 : 0ull;
    const bool ytop = (y == Ly - 1), ybot = (y == 0);
    const uint32_t rp = ytop ? xs * (uint32_t)Ly : row + 1u;
    const uint32_t rm = ybot ? xs * (uint32_t)Ly + (uint32_t)(Ly - 1) : row - 1u;
    const uint64_t Yp = ld64<COH>(sp, rp * RB + qo) ^ (ytop ? seam_mask : 0ull);
    const uint64_t Ym = ld64<COH>(sp, rm * RB + qo) ^ (ybot ? seam_mask : 0ull);
    const uint32_t xstride = (uint32_t)Ly * RB;
    const uint64_t Xm = x > 0 ? ld64<COH>(sp, own - xstride) : 0ull;
    const uint64_t Xp = x < Lx - 1 ? ld64<COH>(sp, own + xstride) : 0ull;
    const uint64_t S = ld64<COH>(sp, own);

    const uint64_t cnt = ((O + Z) + (Yp + Ym)) + (Xm + Xp);
    const int cls = (x == 0 ? 1 : 0) + (x == Lx - 1 ? 2 : 0);
    const int kn = 6 - (x == 0) - (x == Lx - 1);
    const uint64_t idxw = cnt + (S << 3);   // per byte: 8*u + count

    const uint32_t g = ((row * (uint32_t)v.C + 2u * (uint32_t)k) << 1) | (uint32_t)q;
    uint32_t r0[4], r1[4];
    philox10<0u>(g, v.t, v.replica, 0u, v.key0, v.key1, r0);
    philox10<2u>(g, v.t, v.replica, 0u, v.key0, v.key1, r1);

    const uint64_t *tc = sthr + cls * kThrPerClass;
    uint64_t flip = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint32_t e = (uint32_t)(idxw >> (8 * b)) & 0xFFu;
        const uint32_t u = b < 4 ? r0[b] : r1[b - 4];
        flip |= (uint64_t)((uint64_t)u < tc[e & 0xF]) << (8 * b);
    }
    flip &= byte_mask(nv);
    st64<COH>(sp, own, S ^ flip);

    // dB = -2 sum_f s n with s = 2u-1, n = 2 cnt - k;  dM = sum_f (2 - 4u)
    const uint64_t fu = flip & S;
    const int nf = __popcll(flip), nfu = __popcll(fu);
    const uint64_t fm = (flip << 8) - flip, fum = (fu << 8) - fu;
    const int Sf = (int)bytesum64(cnt & fm), Sfu = (int)bytesum64(cnt & fum);
    a.dB += -2 * (4 * Sfu - 2 * kn * nfu - 2 * Sf + kn * nf);
    const int dm = 2 * nf - 4 * nfu;
    a.dM += dm;
    if (x == 0) a.dM1 += dm;
    if (x == Lx - 1) a.dMn += dm;
}

// ---------------------------------------------------------------------------
// bit-packed format: update one 32-bit word (32 same-phase sites).
// Row layout: words [0, Wq) hold even z (z = 2i), words [Wq, 2Wq) odd z.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t bp_bit(const uint32_t *sub, int i)
{
    return (sub[i >> 5] >> (i & 31)) & 1u;
}

template <bool COH>
__device__ __forceinline__ void bp_update_word(const RepView &v, int x, int y, int w, int parity,
                                               const uint64_t *sthr, Acc &a)
{
    const int Lx = v.Lx, Ly = v.Ly, C = v.C, Wq = v.Wq;
    const int nbits = v.Lz >> 1;
    const uint32_t RW = 2u * (uint32_t)Wq;
    const uint32_t row = (uint32_t)x * (uint32_t)Ly + (uint32_t)y;
    auto word = [&](uint32_t i) { return ld32<COH>(v.spins, 4u * i); };
    const int q = (parity + x + y) & 1;
    const uint32_t own = row * RW + (uint32_t)(q * Wq);
    const uint32_t oth = row * RW + (uint32_t)((q ^ 1) * Wq);
    const int nb_here = min(32, nbits - 32 * w);
    const uint32_t vmask = nb_here >= 32 ? 0xFFFFFFFFu : ((1u << nb_here) - 1u);

    const uint32_t S = word(own + w);
    uint32_t zm, zp;
    if (q == 0) {
        // z = 2i: z+1 is odd index i, z-1 is odd index i-1
        const uint32_t O = word(oth + w);
        zp = O;
        const uint32_t carry = (w > 0) ? (word(oth + w - 1) >> 31)
                                       : (word(oth + ((nbits - 1) >> 5)) >> ((nbits - 1) & 31)) & 1u;
        zm = (O << 1) | carry;
    } else {
        // z = 2i+1: z-1 is even index i, z+1 is even index i+1
        const uint32_t E = word(oth + w);
        zm = E;
        const bool lastw = (w == Wq - 1);
        const uint32_t inb = word(oth + (lastw ? 0 : w + 1)) & 1u;
        zp = (E >> 1) | (inb << (lastw ? (nb_here - 1) : 31));
    }

    const uint32_t xs = v.seam_reflect ? (uint32_t)(Lx - 1 - x) : (uint32_t)x;
    const uint32_t seam_mask = v.seam_invert ? 0xFFFFFFFFu : 0u;
    const uint32_t qo = (uint32_t)(q * Wq + w);
    uint32_t yp, ym;
    if (y < Ly - 1) yp = word((row + 1) * RW + qo);
    else yp = word((xs * (uint32_t)Ly) * RW + qo) ^ seam_mask;
    if (y > 0) ym = word((row - 1) * RW + qo);
    else ym = word((xs * (uint32_t)Ly + (uint32_t)(Ly - 1)) * RW + qo) ^ seam_mask;
    const uint32_t xstride = (uint32_t)Ly * RW;
    const uint32_t xm = (x > 0) ? word(own + w - xstride) : 0u;
    const uint32_t xp = (x < Lx - 1) ? word(own + w + xstride) : 0u;

    // bit-sliced count of the six neighbour bits
    const uint32_t s1 = zm ^ zp ^ ym, c1 = (zm & zp) | (ym & (zm ^ zp));
    const uint32_t s2 = yp ^ xm ^ xp, c2 = (yp & xm) | (xp & (yp ^ xm));
    const uint32_t b0 = s1 ^ s2, k0 = s1 & s2;
    const uint32_t b1 = c1 ^ c2 ^ k0, b2 = (c1 & c2) | (k0 & (c1 ^ c2));

    const int cls = (x == 0 ? 1 : 0) + (x == Lx - 1 ? 2 : 0);
    const int k = 6 - (x == 0) - (x == Lx - 1);
    const uint64_t *tc = sthr + cls * kThrPerClass;
    const uint32_t gbase = row * (uint32_t)C + 8u * (uint32_t)w;
    uint32_t F = 0;
    // not unrolled: this path is a small share of the work and must not raise
    // the register count of the kernels it is inlined into
#pragma unroll 1
    for (int g4 = 0; g4 < 8; ++g4) {
        uint32_t rnd[4];
        philox10(((gbase + g4) << 1) | (uint32_t)q, v.t, v.replica, 0u, v.key0, v.key1, rnd);
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int b = 4 * g4 + l;
            const uint32_t e = ((S >> b) & 1u) << 3 | ((b2 >> b) & 1u) << 2 | ((b1 >> b) & 1u) << 1 |
                               ((b0 >> b) & 1u);
            F |= (uint32_t)((uint64_t)rnd[l] < tc[e]) << b;
        }
    }
    F &= vmask;
    st32<COH>(v.spins, 4u * (own + w), S ^ F);

    const uint32_t FU = F & S;
    const int nf = __popc(F), nfu = __popc(FU);
    const int Sf = __popc(F & b0) + 2 * __popc(F & b1) + 4 * __popc(F & b2);
    const int Sfu = __popc(FU & b0) + 2 * __popc(FU & b1) + 4 * __popc(FU & b2);
    a.dB += -2 * (4 * Sfu - 2 * k * nfu - 2 * Sf + k * nf);
    const int dm = 2 * nf - 4 * nfu;
    a.dM += dm;
    if (x == 0) a.dM1 += dm;
    if (x == Lx - 1) a.dMn += dm;
}

// ---------------------------------------------------------------------------
// int8 format, main tiles.
// ---------------------------------------------------------------------------
// The column a thread of a main tile marches: row y (2 .. Ly-2) and column j
// (< ncol columns or words), or false when the thread has none.  A box tile
// is v.ty rows x v.tj columns from (en.y0, en.j0); a linear tile (v.tj = 0)
// is the range [en.y0, en.j0) of the plane's main columns in row-major order,
// one per thread.
__device__ __forceinline__ bool main_column(const RepView &v, const Entry &en, int ncol, int &y, int &j)
{
    if (v.tj > 0) {
        y = en.y0 + v.my_ty;
        j = en.j0 + v.my_tj;
        return v.my_ty < v.ty && y < v.Ly - 1 && j < ncol;
    }
    const int lin = en.y0 + (int)threadIdx.x;
    const int r = (int)((uint32_t)lin / (uint32_t)ncol);
    y = 2 + r;
    j = lin - r * ncol;
    return lin < en.j0;
}

// The view with its draw key (sweep, replica, key words) read from the first
// active lane: the values are the same on every lane, and held in scalar
// registers the Philox round keys cost no vector instructions or registers.
__device__ __forceinline__ RepView uniform_key(const RepView &v)
{
    RepView u = v;
    u.t = __builtin_amdgcn_readfirstlane(v.t);
    u.replica = __builtin_amdgcn_readfirstlane(v.replica);
    u.key0 = __builtin_amdgcn_readfirstlane(v.key0);
    u.key1 = __builtin_amdgcn_readfirstlane(v.key1);
    return u;
}

// Words of one int8 march step, loaded one step ahead of their use.
struct I8Step {
    uint64_t S, yp, ym, xp;   // own column, rows y+1 / y-1 and plane x+1 at the same column
    uint32_t e;               // the z-edge byte of the other sublattice
};

template <bool COH>
__device__ __forceinline__ I8Step i8_load_step(const uint8_t *sp, uint32_t own, uint32_t edge, uint32_t RB,
                                               uint32_t XB, bool has_xp)
{
    I8Step n;
    n.S = ld64<COH>(sp, own);
    n.e = (uint32_t)ld8<COH>(sp, edge);
    n.yp = ld64<COH>(sp, own + RB);
    n.ym = ld64<COH>(sp, own - RB);
    n.xp = has_xp ? ld64<COH>(sp, own + XB) : 0ull;
    return n;
}

// int8 format, main tiles (rows 2 .. Ly-2): a thread owns column k of its
// row's sublattices and marches through the x planes; at plane x it updates
// the 8 sites of sublattice q = (parity + x + y) & 1 in the column.  Of the
// words a step reads, the other sublattice of plane x (O: the z neighbours)
// and the same sublattice of plane x+1 (the x+1 neighbours) are the next
// step's x-1 and other-sublattice words, so they stay in registers; the own
// column, the z-edge byte, rows y+-1 and plane x+2 are loaded one step
// ahead.  None of these bytes is written in this phase.  The per-byte table
// index 8*(8u + cnt) is the byte offset of the site's (thr - 1, packed flip
// change) entry; the plane's class (x = 0, Lx-1) moves the table base.  A
// flip adds its packed (dB, dM) change to a register sum.
template <bool NEVER, bool RAGGED, bool COH>
__device__ __forceinline__ void i8_march(const RepView &v, const Entry &en, int k_lo, int k_hi, int parity,
                                         const Tables *tb, Acc &a)
{
    int y, k;
    if (!main_column(v, en, v.K, y, k)) return;
    const RepView u = uniform_key(v);
    const int Lx = v.Lx, Ly = v.Ly, K = v.K;
    const int Lzh = v.Lz >> 1;
    const uint32_t RB = v.RB, Hp = v.Hp;
    const uint32_t XB = (uint32_t)Ly * RB;   // bytes of one x plane
    const uint32_t co = 8u * (uint32_t)k;
    const bool last = (k == K - 1);
    const int nv = RAGGED && last ? Lzh - 8 * (K - 1) : 8;
    // the z-edge byte: own q = 0 needs odd byte 8k-1 (Lzh-1 for k = 0) at
    // bit 0; own q = 1 needs even byte 8k+8 (byte 0 for the last column) at
    // byte nv-1
    const uint32_t e0 = Hp + (k > 0 ? co - 1u : (uint32_t)(Lzh - 1));
    const uint32_t e1 = last ? 0u : co + 8u;
    const uint32_t esh = RAGGED ? 8u * (uint32_t)(nv - 1) : 24u;   // in the high word unless ragged
    const int x0 = en.x0 + k_lo;
    const int x1 = min(en.x0 + k_hi, Lx);
    int q = (parity + x0 + y) & 1;
    uint32_t rw = ((uint32_t)x0 * (uint32_t)Ly + (uint32_t)y) * RB;   // byte offset of row (x, y)
    const uint32_t gstep = 2u * (uint32_t)Ly * (uint32_t)v.C;
    uint32_t g = ((((uint32_t)x0 * (uint32_t)Ly + (uint32_t)y) * (uint32_t)v.C + 2u * (uint32_t)k) << 1) |
                 (uint32_t)q;

    auto own_of = [&](uint32_t r, int qq) { return r + (qq ? Hp : 0u) + co; };
    auto edge_of = [&](uint32_t r, int qq) { return r + (qq ? e1 : e0); };
    uint64_t O = ld64<COH>(v.spins, own_of(rw, q ^ 1));
    uint64_t xm = x0 > 0 ? ld64<COH>(v.spins, own_of(rw, q) - XB) : 0ull;
    I8Step cur = i8_load_step<COH>(v.spins, own_of(rw, q), edge_of(rw, q), RB, XB, x0 < Lx - 1);
    // the surface planes x = 0 and Lx-1 can only be the first and last step
    // of a march: they run apart from the bulk steps (their own tables and
    // M1 / Mn sums), the bulk steps use the bulk class's table
    int dsum = 0, dsurf1 = 0, dsurfn = 0;
    int x = x0;
    auto step = [&](auto surface) {
        constexpr bool SURF = decltype(surface)::value;
        const uint32_t own = own_of(rw, q);
        I8Step nxt;
        const bool more = x + 1 < x1;
        if (more) nxt = i8_load_step<COH>(v.spins, own_of(rw + XB, q ^ 1), edge_of(rw + XB, q ^ 1), RB, XB, x + 2 < Lx);
        // bytes hold 0/1 and their sums stay below 8, so no carry crosses a
        // byte: each 32-bit half of the column is summed on its own
        const uint32_t ol = (uint32_t)O, oh = (uint32_t)(O >> 32);
        uint32_t zl, zh;
        if (q) {
            // z+1: the other sublattice one byte up, the edge byte on top
            zl = __builtin_amdgcn_alignbit(oh, ol, 8);
            zh = oh >> 8;
            if (RAGGED) {
                const uint64_t eb = (uint64_t)cur.e << esh;
                zl |= (uint32_t)eb;
                zh |= (uint32_t)(eb >> 32);
            } else {
                zh |= cur.e << 24;
            }
        } else {
            // z-1: the other sublattice one byte down, the edge byte at the bottom
            zl = (ol << 8) | cur.e;
            zh = __builtin_amdgcn_alignbit(oh, ol, 24);
        }
        const uint32_t sl = (uint32_t)cur.S, sh = (uint32_t)(cur.S >> 32);
        const uint32_t cl = ((ol + zl) + ((uint32_t)cur.yp + (uint32_t)cur.ym)) + ((uint32_t)xm + (uint32_t)cur.xp);
        const uint32_t ch = ((oh + zh) + ((uint32_t)(cur.yp >> 32) + (uint32_t)(cur.ym >> 32))) +
                            ((uint32_t)(xm >> 32) + (uint32_t)(cur.xp >> 32));
        // per byte 8 (8u + cnt): the entry's byte offset in its class's table
        const uint32_t il = (cl + (sl << 3)) << 3;
        const uint32_t ih = (ch + (sh << 3)) << 3;
        const int cls = SURF ? (x == 0 ? 1 : 0) + (x == Lx - 1 ? 2 : 0) : 0;
        const char *tdc = (const char *)(tb->td + cls * kThrPerClass);
        const char *thc = (const char *)(tb->thr + cls * kThrPerClass);
        uint32_t r0[4], r1[4];
        philox10<0u>(g, u.t, u.replica, 0u, u.key0, u.key1, r0);
        philox10<2u>(g, u.t, u.replica, 0u, u.key0, u.key1, r1);
        uint32_t fl = 0, fh = 0;
        int step = 0;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint32_t w = b < 4 ? il : ih;
            const uint32_t off = (w >> (8 * (b & 3))) & 0xFFu;
            const uint32_t u = b < 4 ? r0[b] : r1[b - 4];
            const TD t = *(const TD *)(tdc + off);
            bool acc;
            if (NEVER) acc = (uint64_t)u < *(const uint64_t *)(thc + off);
            else acc = u <= t.thr_m1;
            if (RAGGED) acc = acc && (b < nv);
            step += acc ? t.dpack : 0;
            if (b < 4) fl |= (acc ? 1u : 0u) << (8 * b);
            else fh |= (acc ? 1u : 0u) << (8 * (b - 4));
        }
        st64<COH>(v.spins, own, cur.S ^ (((uint64_t)fh << 32) | fl));
        dsum += step;
        if (SURF) {
            if (x == 0) dsurf1 = step;
            if (x == Lx - 1) dsurfn = step;
        }
        // the next plane: its x-1 word is this plane's other sublattice, its
        // other-sublattice word is this plane's x+1 word
        xm = O;
        O = cur.xp;
        if (more) cur = nxt;
        rw += XB;
        g += gstep;
        g ^= 1u;
        q ^= 1;
        ++x;
    };
    if (x0 == 0 && x0 < x1) step(std::true_type{});
    const int xb1 = min(x1, Lx - 1);
    while (x < xb1) step(std::false_type{});
    if (x < x1) step(std::true_type{});
    // packed sums: dB in the low 16 bits (|sum| < 2^15 for <= kMaxMarch planes of 8 sites)
    const int dB = (int)(int16_t)(dsum & 0xFFFF), dM = (dsum - dB) >> 16;
    a.dB += dB;
    a.dM += dM;
    const int dB1 = (int)(int16_t)(dsurf1 & 0xFFFF), dBn = (int)(int16_t)(dsurfn & 0xFFFF);
    a.dM1 += (dsurf1 - dB1) >> 16;
    a.dMn += (dsurfn - dBn) >> 16;
}

// Spreads the low 8 bits of x to bits 0, 4, 8, ..., 28 (one site per nibble).
__device__ __forceinline__ uint32_t spread_nibbles(uint32_t x)
{
    x &= 0xFFu;
    x = (x | (x << 12)) & 0x000F000Fu;
    x = (x | (x << 6)) & 0x03030303u;
    x = (x | (x << 3)) & 0x11111111u;
    return x;
}

// bit-packed format, main tiles (rows 2 .. Ly-2): a thread owns word w of its
// row's sublattices and marches through the x planes; at plane x it updates
// the sublattice of the phase's parity q (q alternates with x).  Of the words
// a step reads, the other sublattice of plane x (O) and the same sublattice
// of plane x+1 (xp) are the next step's x-1 and other-sublattice words, so
// they stay in registers; the rest (own word, z-edge word, y neighbours,
// plane x+2) are loaded one step ahead.  None of these words is written in
// this phase.  Neighbour counts are bit-sliced.  On bulk planes the 4-bit
// table indices 8u + cnt of the site pairs (j, j+16) are gathered into bytes
// (bp_flips_pairs); surface planes and never-accepted moves gather them into
// nibbles and look up one site at a time (bp_flips).
struct BpStep {
    uint32_t S, A, yp, ym, xp;
};

template <bool COH>
__device__ __forceinline__ BpStep bp_load_step(const uint8_t *sp, uint32_t own, uint32_t edge, uint32_t RWB,
                                               uint32_t XB, bool has_xp)
{
    BpStep n;
    n.S = ld32<COH>(sp, own);
    n.A = ld32<COH>(sp, edge);
    n.yp = ld32<COH>(sp, own + RWB);
    n.ym = ld32<COH>(sp, own - RWB);
    n.xp = has_xp ? ld32<COH>(sp, own + XB) : 0u;
    return n;
}

// Shifts the reject bits (thr - 1 < r) of eight sites into two words:
// lo = 2 lo + reject(site of t[l].x, r0[l]) and hi likewise with t[l].y and
// r1[l], for l = 3, 2, 1, 0 (FIRST: lo and hi start from 0).  Each compare
// writes a carry register that an add-with-carry (x + x + carry) consumes:
// two instructions per site.  Three carry registers rotate so that each is
// read two or more instructions after the compare writes it, the wait gfx950
// needs between a VALU write of a scalar register and a VALU read of it.
// VALU instructions only.
#define ISLF_REJECT8_ASM(LO0, HI0)                                                                                     \
    "v_cmp_lt_u32_e64 %[a], %[t3x], %[r03]\n\t"                                                                         \
    "v_cmp_lt_u32_e64 %[b], %[t3y], %[r13]\n\t"                                                                         \
    "v_cmp_lt_u32_e32 vcc, %[t2x], %[r02]\n\t"                                                                          \
    "v_addc_co_u32_e64 %[lo], %[a], " LO0 ", " LO0 ", %[a]\n\t"                                                         \
    "v_addc_co_u32_e64 %[hi], %[b], " HI0 ", " HI0 ", %[b]\n\t"                                                         \
    "v_cmp_lt_u32_e64 %[a], %[t2y], %[r12]\n\t"                                                                         \
    "v_addc_co_u32_e32 %[lo], vcc, %[lo], %[lo], vcc\n\t"                                                               \
    "v_cmp_lt_u32_e64 %[b], %[t1x], %[r01]\n\t"                                                                         \
    "v_cmp_lt_u32_e32 vcc, %[t1y], %[r11]\n\t"                                                                          \
    "v_addc_co_u32_e64 %[hi], %[a], %[hi], %[hi], %[a]\n\t"                                                             \
    "v_addc_co_u32_e64 %[lo], %[b], %[lo], %[lo], %[b]\n\t"                                                             \
    "v_cmp_lt_u32_e64 %[a], %[t0x], %[r00]\n\t"                                                                         \
    "v_addc_co_u32_e32 %[hi], vcc, %[hi], %[hi], vcc\n\t"                                                               \
    "v_cmp_lt_u32_e64 %[b], %[t0y], %[r10]\n\t"                                                                         \
    "v_addc_co_u32_e64 %[lo], %[a], %[lo], %[lo], %[a]\n\t"                                                             \
    "s_nop 0\n\t"                                                                                                       \
    "v_addc_co_u32_e64 %[hi], %[b], %[hi], %[hi], %[b]"
#define ISLF_REJECT8_IN                                                                                                \
    [t3x] "v"(t[3].x), [t3y] "v"(t[3].y), [t2x] "v"(t[2].x), [t2y] "v"(t[2].y), [t1x] "v"(t[1].x),                   \
        [t1y] "v"(t[1].y), [t0x] "v"(t[0].x), [t0y] "v"(t[0].y), [r03] "v"(r0[3]), [r13] "v"(r1[3]),                  \
        [r02] "v"(r0[2]), [r12] "v"(r1[2]), [r01] "v"(r0[1]), [r11] "v"(r1[1]), [r00] "v"(r0[0]), [r10] "v"(r1[0])

template <bool FIRST>
__device__ __forceinline__ void reject_bits8(uint32_t &lo, uint32_t &hi, const uint2 t[4], const uint32_t r0[4],
                                             const uint32_t r1[4])
{
    uint64_t ca, cb;
    if (FIRST)
        asm(ISLF_REJECT8_ASM("0", "0")
            : [lo] "=&v"(lo), [hi] "=&v"(hi), [a] "=&s"(ca), [b] "=&s"(cb)
            : ISLF_REJECT8_IN
            : "vcc");
    else
        asm(ISLF_REJECT8_ASM("%[lo]", "%[hi]")
            : [lo] "+v"(lo), [hi] "+v"(hi), [a] "=&s"(ca), [b] "=&s"(cb)
            : ISLF_REJECT8_IN
            : "vcc");
}
#undef ISLF_REJECT8_ASM
#undef ISLF_REJECT8_IN

// Accept bits of the 32 sites of one word, bulk class, thresholds read from
// the pair table for the neighbouring sites (2m, 2m+1).  Byte m of w[k]
// interleaves the index bits e = 8u + cnt of sites 8m + 2k and 8m + 2k + 1:
// its 2-bit fields are bits (2k, 2k+1) of byte m of the planes b0, b1, b2
// and S, placed by shifts and bitfield inserts (the four fields cover every
// bit of a byte).  Philox call c (counter gq + 2c) draws for sites
// 4c .. 4c+3.
__device__ __forceinline__ uint32_t bp_flips_pairs(uint32_t S, uint32_t b2, uint32_t b1, uint32_t b0, uint32_t gq,
                                                   const RepView &v, const Tables *tb)
{
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t acc = b0 >> (2 * k);
        acc = __builtin_amdgcn_bitop3_b32(0x0C0C0C0Cu, k == 0 ? b1 << 2 : b1 >> (2 * k - 2), acc, 0xCA);
        acc = __builtin_amdgcn_bitop3_b32(0x30303030u, k <= 2 ? b2 << (4 - 2 * k) : b2 >> 2, acc, 0xCA);
        w[k] = __builtin_amdgcn_bitop3_b32(0xC0C0C0C0u, S << (6 - 2 * k), acc, 0xCA);
    }
    // sites are visited from the top down (g = 3 .. 0, l = 3 .. 0), so that
    // the shifted-in reject bits end at their site's position; the
    // thresholds are read before the draws so that the LDS latency overlaps
    // Philox
    uint32_t rlo, rhi;
    auto group = [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        // sites 4g .. 4g+3: byte g/2 of w[2(g&1)] and w[2(g&1)+1]; sites
        // 4g+16 .. 4g+19: byte 2 + g/2 of the same words
        constexpr int k = 2 * (g & 1), lo = 8 * (g >> 1), hi = lo + 16;
        const uint2 l0 = tb->pair[(w[k] >> lo) & 0xFFu], l1 = tb->pair[(w[k + 1] >> lo) & 0xFFu];
        const uint2 h0 = tb->pair[(w[k] >> hi) & 0xFFu], h1 = tb->pair[(w[k + 1] >> hi) & 0xFFu];
        // t[l]: thresholds of site 4g+l (x) and 4g+16+l (y)
        const uint2 t[4] = {make_uint2(l0.x, h0.x), make_uint2(l0.y, h0.y), make_uint2(l1.x, h1.x),
                            make_uint2(l1.y, h1.y)};
        uint32_t r0[4], r1[4];
        philox10<2u * g>(gq, v.t, v.replica, 0u, v.key0, v.key1, r0);
        philox10<2u * (g + 4)>(gq, v.t, v.replica, 0u, v.key0, v.key1, r1);
        reject_bits8<g == 3>(rlo, rhi, t, r0, r1);
    };
    group(std::integral_constant<int, 3>{});
    group(std::integral_constant<int, 2>{});
    group(std::integral_constant<int, 1>{});
    group(std::integral_constant<int, 0>{});
    return ~(rlo | (rhi << 16));
}

// Accept bits of the 32 sites of one word, any class: eight Philox draws
// (counters gq + 2i, i = 0..7, four sites each); the 4-bit table index
// 8u + cnt of every site is gathered into nibbles (eight sites per word) and
// looked up one site at a time (64-bit compare under NEVER).
template <bool NEVER>
__device__ __forceinline__ uint32_t bp_flips(uint32_t S, uint32_t b2, uint32_t b1, uint32_t b0, uint32_t gq,
                                             const RepView &v, const Tables *tb, int cls)
{
    const TD *tdc = tb->td + cls * kThrPerClass;
    const uint64_t *thc = tb->thr + cls * kThrPerClass;
    uint32_t F = 0;
    // one byte of sites per iteration, not unrolled: unrolling lets the
    // compiler keep all 32 draws live and costs occupancy
#pragma unroll 1
    for (int h = 0; h < 4; ++h) {
        // eight sites 8h .. 8h+7: nibble i holds 8u + cnt of site 8h+i
        const int sh = 8 * h;
        const uint32_t nib = (spread_nibbles(S >> sh) << 3) | (spread_nibbles(b2 >> sh) << 2) |
                             (spread_nibbles(b1 >> sh) << 1) | spread_nibbles(b0 >> sh);
        uint32_t Fh = 0;
#pragma unroll
        for (int g2 = 0; g2 < 2; ++g2) {
            uint32_t rnd[4];
            philox10(gq + 2u * (uint32_t)(2 * h + g2), v.t, v.replica, 0u, v.key0, v.key1, rnd);
            {
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    const int i = 4 * g2 + l;
                    const uint32_t e = (nib >> (4 * i)) & 0xFu;
                    bool acc;
                    if (NEVER) acc = (uint64_t)rnd[l] < thc[e];
                    else acc = rnd[l] <= tdc[e].thr_m1;
                    Fh |= (uint32_t)acc << i;
                }
            }
        }
        F |= Fh << sh;
    }
    return F;
}

template <bool NEVER, bool COH>
__device__ __forceinline__ void bp_march(const RepView &v, const Entry &en, int k_lo, int k_hi, int parity,
                                         const Tables *tb, Acc &a)
{
    int y, w;
    if (!main_column(v, en, v.Wq, y, w)) return;
    const RepView u = uniform_key(v);
    const int Lx = v.Lx, Ly = v.Ly, C = v.C, Wq = v.Wq;
    const int nbits = v.Lz >> 1;
    const uint32_t SB = 4u * (uint32_t)Wq;    // bytes of one sublattice row
    const uint32_t RWB = 2u * SB;             // bytes of one row
    const uint32_t XB = (uint32_t)Ly * RWB;   // bytes of one x plane
    const int nb_here = min(32, nbits - 32 * w);
    const uint32_t vmask = nb_here >= 32 ? 0xFFFFFFFFu : ((1u << nb_here) - 1u);
    // z edges: an even-z word (q = 0) needs bit 31 of odd word w-1 (the last
    // odd bit when w = 0); an odd-z word (q = 1) needs bit 0 of even word w+1
    // (of word 0 for the last word, placed at bit nb_here-1)
    const bool lastw = (w == Wq - 1);
    const uint32_t e0 = 4u * (uint32_t)(w > 0 ? w - 1 : (nbits - 1) >> 5);
    const uint32_t e1 = 4u * (uint32_t)(lastw ? 0 : w + 1);
    const uint32_t csh0 = w > 0 ? 31u : (uint32_t)((nbits - 1) & 31);
    const uint32_t zsh1 = lastw ? (uint32_t)(nb_here - 1) : 31u;
    const int x0 = en.x0 + k_lo;
    const int x1 = min(en.x0 + k_hi, Lx);
    int q = (parity + x0 + y) & 1;
    // byte offset of row (x, y), word w of sublattice 0
    uint32_t rw = ((uint32_t)x0 * (uint32_t)Ly + (uint32_t)y) * RWB + 4u * (uint32_t)w;
    const uint32_t gstep = 2u * (uint32_t)Ly * (uint32_t)C;
    uint32_t gq = ((((uint32_t)x0 * (uint32_t)Ly + (uint32_t)y) * (uint32_t)C + 8u * (uint32_t)w) << 1) |
                  (uint32_t)q;

    auto own_of = [&](uint32_t r, int qq) { return r + (qq ? SB : 0u); };
    auto edge_of = [&](uint32_t r, int qq) { return r - 4u * (uint32_t)w + (qq ? e1 : SB + e0); };
    uint32_t O = ld32<COH>(v.spins, own_of(rw, q ^ 1));
    uint32_t xm = (x0 > 0) ? ld32<COH>(v.spins, own_of(rw, q) - XB) : 0u;
    BpStep cur = bp_load_step<COH>(v.spins, own_of(rw, q), edge_of(rw, q), RWB, XB, x0 < Lx - 1);
    // per-thread sums over the flipped sites of the march: NF = flips, NFU =
    // flips of up spins, A0..A2 = bit planes of a' = c (up) or 7 - c (down),
    // c = up neighbours; KDM = sum of (6 - k) dm over the surface planes
    int NF = 0, NFU = 0, A0 = 0, A1 = 0, A2 = 0, KDM = 0;
    // one step at plane x; the surface planes x = 0 and Lx-1 can only be the
    // first and last step of a march and run apart from the bulk steps (their
    // own tables, fewer neighbours, the M1 / Mn sums)
    int x = x0;
    auto step = [&](auto surface) {
        constexpr bool SURF = decltype(surface)::value;
        const uint32_t own = own_of(rw, q);
        BpStep nxt;
        const bool more = x + 1 < x1;
        if (more) nxt = bp_load_step<COH>(v.spins, own_of(rw + XB, q ^ 1), edge_of(rw + XB, q ^ 1), RWB, XB, x + 2 < Lx);
        const uint32_t S = cur.S;
        const uint32_t zm = q ? O : ((O << 1) | ((cur.A >> csh0) & 1u));
        const uint32_t zp = q ? ((O >> 1) | ((cur.A & 1u) << zsh1)) : O;
        const uint32_t ym = cur.ym, yp = cur.yp, xp = cur.xp;

        const uint32_t s1 = zm ^ zp ^ ym, c1 = (zm & zp) | (ym & (zm ^ zp));
        const uint32_t s2 = yp ^ xm ^ xp, c2 = (yp & xm) | (xp & (yp ^ xm));
        const uint32_t b0 = s1 ^ s2, k0 = s1 & s2;
        const uint32_t b1 = c1 ^ c2 ^ k0, b2 = (c1 & c2) | (k0 & (c1 ^ c2));

        uint32_t F;
        if (SURF) F = bp_flips<NEVER>(S, b2, b1, b0, gq, u, tb, (x == 0 ? 1 : 0) + (x == Lx - 1 ? 2 : 0));
        else if (NEVER) F = bp_flips<true>(S, b2, b1, b0, gq, u, tb, 0);
        else F = bp_flips_pairs(S, b2, b1, b0, gq, u, tb);
        F &= vmask;
        st32<COH>(v.spins, own, S ^ F);
        const uint32_t FU = F & S;
        NF += __popc(F);
        NFU += __popc(FU);
        // F & ~(b ^ S): the bit planes of a' on the flipped sites
        A0 += __popc(__builtin_amdgcn_bitop3_b32(F, b0, S, 0x90));
        A1 += __popc(__builtin_amdgcn_bitop3_b32(F, b1, S, 0x90));
        A2 += __popc(__builtin_amdgcn_bitop3_b32(F, b2, S, 0x90));
        if (SURF) {
            const int dm = 2 * __popc(F) - 4 * __popc(FU);
            if (x == 0) a.dM1 += dm;
            if (x == Lx - 1) a.dMn += dm;
            KDM += ((x == 0) + (x == Lx - 1)) * dm;
        }
        // the next plane: its x-1 word is this plane's other sublattice, its
        // other-sublattice word is this plane's x+1 word
        xm = O;
        O = xp;
        if (more) cur = nxt;
        rw += XB;
        gq += gstep;
        gq ^= 1u;
        q ^= 1;
        ++x;
    };
    if (x0 == 0 && x0 < x1) step(std::true_type{});
    const int xb1 = min(x1, Lx - 1);
    while (x < xb1) step(std::false_type{});
    if (x < x1) step(std::true_type{});
    // a flip of spin s = 2u - 1 with c of its k neighbours up changes B by
    // -2 s (2c - k) = -2 (2a' - k) (up) or -2 (2a' + k - 14) (down); summed
    // with k = 6 - (6 - k): -4 A + 16 NF - 4 NFU + KDM, A = A0 + 2 A1 + 4 A2
    a.dB += -4 * (A0 + 2 * A1 + 4 * A2) + 16 * NF - 4 * NFU + KDM;
    a.dM += 2 * NF - 4 * NFU;
}

// ---------------------------------------------------------------------------
// Sweep schedule.  The four phases of sweep t run in two launches:
//   A(t): phase 3 of sweep t-1 on row 0, then phase 0 of sweep t;
//   B(t): phase 1 of sweep t, then phase 2 of sweep t on row 0;
// and a final launch F runs phase 3 of the last sweep.  Rows 2 .. Ly-2 are
// done by main (marching) tiles.  Rows Ly-1, 0 and 1 belong to seam-slab
// tiles: a slab tile owns a set of x planes closed under x -> Lx-1-x and a
// range of z columns, and runs its two stages with one workgroup barrier in
// between.  Every input a stage reads is either written earlier by the same
// workgroup or not written by anybody during that launch:
//  - phase 3 (row 0) reads row-0 phase-2 sites (written only in B) and rows
//    1 / Ly-1 before this launch's phase 0 (whose sites it shares rows with
//    are updated by the same slab tile, after the barrier);
//  - phase 0 on rows 1 / Ly-1 reads row 0 at the same z and x or Lx-1-x,
//    both in the tile, after its phase-3 stage;
//  - phase 1 on rows 1 / Ly-1 reads row-0 phase-2 sites before their update
//    (same tile, later stage) and phase-0 sites (not written in B);
//  - phase 2 on row 0 reads rows 1 / Ly-1 after the tile's phase-1 stage.
// Main tiles never read row 0.  The record of sweep t-1 is folded by block 0
// of B(t) (all of its phases are complete by then; B(t) only adds to the
// other accumulator half), the last sweep's by the last block of F.
// A slab entry is (rep, first x pair, number of pairs, first column,
// number of columns) in the fields (rep, x0, y0, j0, nsteps).
// ---------------------------------------------------------------------------
// One wave folds the spread partial sums of sweep t of one replica into its
// running observables and record (slots read and cleared atomically; COH:
// the running sums are read and written device-coherently).
template <bool COH>
__device__ __forceinline__ void fold_sweep(const RepDesc &d, RepState &sr, uint32_t t, int lane)
{
    long long *slot = d.acc + ((size_t)(t & 1) * kAccSlots + lane) * 4;
    long long v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (long long)atomicExch((unsigned long long *)&slot[k], 0ull);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    }
    if (lane == 0) {
        long long c[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            c[k] = COH ? __hip_atomic_load(&sr.cur[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : sr.cur[k];
            c[k] += v[k];
            if (COH) __hip_atomic_store(&sr.cur[k], c[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else sr.cur[k] = c[k];
        }
        islf_obs o;
        o.B = c[0];
        o.M = c[1];
        o.M1 = c[2];
        o.Mn = c[3];
        d.rec[t % d.cap] = o;
    }
}

// Wave w of the grid (blockIdx * 4 + wave) folds sweep st.t + s of the listed
// replicas w, w + 4*grid, ...; with `advance` it then moves their sweep
// counters on by that much.  Waves only: no workgroup barrier.
template <bool COH>
__device__ __forceinline__ void fold_waves(const RepDesc *__restrict__ descs, RepState *__restrict__ st,
                                           const int *__restrict__ reps, int n_reps, uint32_t s, uint32_t advance)
{
    const int lane = threadIdx.x & 63;
    const int per_block = kBlock / 64;
    for (int i = blockIdx.x * per_block + (threadIdx.x >> 6); i < n_reps; i += gridDim.x * per_block) {
        const int r = reps[i];
        fold_sweep<COH>(descs[r], st[r], st[r].t + s, lane);
        if (advance && lane == 0) st[r].t += advance;
    }
}

// Updates of one slab stage: `phase` decides the rows (0/1: rows 1 and Ly-1,
// one row when Ly = 2; 2/3: row 0) and the parity; the x pairs and the
// columns come from the entry.  Sites of one phase are never neighbours, so
// the tasks of a stage are independent.
template <int FMT, bool COH>
__device__ __forceinline__ void slab_stage(const RepView &v, const Entry &en, int phase, const Tables *tb, Acc &a)
{
    const int Lx = v.Lx, Ly = v.Ly;
    const int p0 = en.x0, np = en.y0, j0 = en.j0, nj = en.nsteps;
    const int rows = phase >= 2 ? 1 : (Ly == 2 ? 1 : 2);
    const int nx = 2 * np;
    const int ntask = rows * nx * nj;
    for (int k = threadIdx.x; k < ntask; k += kBlock) {
        const int jj = k % nj;
        const int rest = k / nj;
        const int xi = rest % nx, ri = rest / nx;
        const int p = p0 + (xi >> 1);
        const int x = (xi & 1) ? Lx - 1 - p : p;
        if ((xi & 1) && x == p) continue;   // the middle plane of an odd Lx pairs with itself
        const int y = phase >= 2 ? 0 : (ri == 0 ? 1 : Ly - 1);
        if (FMT == ISLF_SPIN_INT8) i8_update_col<COH>(v, x, y, j0 + jj, phase & 1, tb->thr, a);
        else bp_update_word<COH>(v, x, y, j0 + jj, phase & 1, tb->thr, a);
    }
}

// One slab entry of launch KIND for sweep st.t + s; ends with a workgroup
// barrier (in the last flush).
// Stages replica rep's tables in LDS unless they are there already.  key
// (uniform, kept by the caller across items and, in the persistent kernels,
// across stages) names what LDS holds: 2 rep + 1 with the pair table, 2 rep
// without, -1 nothing.  A reload follows a workgroup barrier of the caller
// (the previous item's flush, or a grid barrier), so no wave still reads the
// old tables.
template <bool PAIRS>
__device__ __forceinline__ void ensure_tables(const RepDesc *__restrict__ descs, int rep, Tables *tb, int &key)
{
    if (key == 2 * rep + 1 || (!PAIRS && key == 2 * rep)) return;
    load_tables<PAIRS>(descs[rep], tb);
    __syncthreads();
    key = 2 * rep + (PAIRS ? 1 : 0);
}

template <int FMT, int KIND, bool COH>
__device__ __forceinline__ void slab_entry(const RepDesc *__restrict__ descs, const RepState *__restrict__ st,
                                           const Entry &en, uint32_t s, uint32_t flags, Tables *tb, int &tb_key)
{
    const RepView v = load_view(descs, st, en.rep, s);
    ensure_tables<false>(descs, en.rep, tb, tb_key);
    const int slot = blockIdx.x & (kAccSlots - 1);
    Acc a = {0, 0, 0, 0};
    if (KIND == KIND_A) {
        if (flags & FLAG_PREV) {
            RepView vp = v;
            vp.t = v.t - 1;
            slab_stage<FMT, COH>(vp, en, 3, tb, a);
            flush_acc(a, v.acc, vp.t, slot);   // its barrier also orders the two stages
        }
        slab_stage<FMT, COH>(v, en, 0, tb, a);
        flush_acc(a, v.acc, v.t, slot);
    } else if (KIND == KIND_B) {
        slab_stage<FMT, COH>(v, en, 1, tb, a);
        flush_acc(a, v.acc, v.t, slot);
        slab_stage<FMT, COH>(v, en, 2, tb, a);
        flush_acc(a, v.acc, v.t, slot);
    } else {
        slab_stage<FMT, COH>(v, en, 3, tb, a);
        flush_acc(a, v.acc, v.t, slot);
    }
}

// One main tile piece (rows 2 .. Ly-2), x steps [k_lo, k_hi), of launch A
// (phase 0) or B (phase 1), with the replica's view and tables in place;
// adds its changes of the observables to a.
template <int FMT, int KIND, bool COH>
__device__ __forceinline__ void main_piece(const RepView &v, const Entry &en, int k_lo, int k_hi, const Tables *tb,
                                           Acc &a)
{
    const int parity = KIND == KIND_A ? 0 : 1;
    if (FMT == ISLF_SPIN_INT8) {
        const bool ragged = (v.Lz & 15) != 0;   // a sublattice row ends in a partial column
        if (v.never) {
            if (ragged) i8_march<true, true, COH>(v, en, k_lo, k_hi, parity, tb, a);
            else i8_march<true, false, COH>(v, en, k_lo, k_hi, parity, tb, a);
        } else {
            if (ragged) i8_march<false, true, COH>(v, en, k_lo, k_hi, parity, tb, a);
            else i8_march<false, false, COH>(v, en, k_lo, k_hi, parity, tb, a);
        }
    } else {
        if (v.never) bp_march<true, COH>(v, en, k_lo, k_hi, parity, tb, a);
        else bp_march<false, COH>(v, en, k_lo, k_hi, parity, tb, a);
    }
}

// Workgroup b of a launch plan runs items [first[b'], first[b'+1]) in order,
// where b' spreads consecutive plan blocks over the eight XCDs' dispatch
// order so that each XCD (and its L2) works on a contiguous run of tiles.
__device__ __forceinline__ int plan_block()
{
    // workgroups go to the 8 XCDs in turn (block b to XCD b mod 8); XCD x
    // takes the contiguous run of plan slots starting at x*q + min(x, r)
    // (G = 8q + r), so that neighbouring pieces share its L2
    const int b = blockIdx.x, G = gridDim.x;
    const int x = b & 7, q = G >> 3, r = G & 7;
    return x * q + min(x, r) + (b >> 3);
}

template <int FMT, int KIND, bool COH>
__device__ __forceinline__ void run_items(const RepDesc *__restrict__ descs, const RepState *__restrict__ st,
                                          const Entry *__restrict__ items, int i0, int i1, uint32_t s,
                                          uint32_t flags, Tables *tb, int &tb_key)
{
    // a workgroup's slab items come before its main pieces; consecutive main
    // pieces of one replica share the loaded view and tables and one flush
    // of their summed changes
    int i = i0;
    for (; i < i1; ++i) {
        const Entry en = items[i];
        if (en.kind != ITEM_SLAB) break;
        slab_entry<FMT, KIND, COH>(descs, st, en, s, flags, tb, tb_key);
    }
    if (KIND == KIND_F) return;
    const int slot = blockIdx.x & (kAccSlots - 1);
    int cur = -1;
    RepView v;
    Acc a = {0, 0, 0, 0};
    for (; i < i1; ++i) {
        const Entry en = items[i];
        if (en.rep != cur) {
            if (cur >= 0) flush_acc(a, v.acc, v.t, slot);   // its barrier frees the tables
            v = load_view(descs, st, en.rep, s);
            ensure_tables<FMT == ISLF_SPIN_BITPACK>(descs, en.rep, tb, tb_key);
            cur = en.rep;
        }
        main_piece<FMT, KIND, COH>(v, en, 0, en.nsteps, tb, a);
    }
    if (cur >= 0) flush_acc(a, v.acc, v.t, slot);
}

// Launches A, B and F of sweep st.t + s over a launch plan (slab items come
// first in the plan, so F only launches the blocks that hold them).  With
// FLAG_FOLD, waves of B first fold the previous sweep's record.
template <int FMT, int KIND>
__global__ __launch_bounds__(kBlock) void k_sweep(const RepDesc *__restrict__ descs, RepState *__restrict__ st,
                                                  const Entry *__restrict__ items, const int *__restrict__ first,
                                                  const int *__restrict__ reps, int n_reps, uint32_t s,
                                                  uint32_t flags)
{
    __shared__ Tables tb;
    if (KIND == KIND_B && (flags & FLAG_FOLD)) fold_waves<false>(descs, st, reps, n_reps, s - 1, 0u);
    const int b = plan_block();
    int tb_key = -1;
    run_items<FMT, KIND, false>(descs, st, items, first[b], first[b + 1], s, flags, &tb, tb_key);
}

// Closes a run of sweeps: folds sweep st.t + s and advances the counters.
__global__ __launch_bounds__(kBlock) void k_fold(const RepDesc *__restrict__ descs, RepState *__restrict__ st,
                                                 const int *__restrict__ reps, int n_reps, uint32_t s,
                                                 uint32_t advance)
{
    fold_waves<false>(descs, st, reps, n_reps, s, advance);
}

// ---------------------------------------------------------------------------
// Persistent form: the same schedule inside one cooperative launch, with a
// bounded two-level grid barrier in place of each launch boundary.
// ---------------------------------------------------------------------------
// Polls a barrier word (a device-coherent load).
__device__ __forceinline__ unsigned long long sync_load(unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits (bounded) until *p >= target; false on time-out or a raised error
// word (checked before the first poll too, so that once one block has given
// up, every later barrier of the launch gives up at once).
__device__ __forceinline__ bool sync_wait(GridSync *sync, unsigned long long *p, unsigned long long target)
{
    unsigned long spins = 0;
    while (true) {
        if (sync_load(&sync->error.v)) return false;
        if (sync_load(p) >= target) return true;
        __builtin_amdgcn_s_sleep(1);
        if (++spins > (1ul << 22)) {
            atomicAdd(&sync->error.v, 1ull);
            return false;
        }
    }
}

// Barrier number k (= passed) of a launch: two-level arrival, see GridSync.
// Everything the persistent kernel's blocks share across a barrier (lattice
// words, running sums, accumulator slots, barrier words) is accessed
// device-coherently: coherent loads and stores or device-scope atomics, none
// of which leaves a line that another XCD could miss in its L2 or find stale
// in its own.  The barrier therefore orders them by completion alone: every
// wave waits until its memory operations are complete before the workgroup
// meets, thread 0 arrives with a device-scope atomic once they all are, and
// no wave issues a load of the next phase before thread 0 has seen the last
// arrival.  The fences are workgroup-scope (they order the compiler and the
// workgroup): device-scope fences would write back and invalidate the whole
// L2 at each barrier.
__device__ bool grid_barrier(GridSync *sync, unsigned long long nblocks, unsigned long long &passed)
{
    __builtin_amdgcn_s_waitcnt(0);   // all counters: this wave's loads and stores are complete
    __syncthreads();
    __shared__ int ok;
    if (threadIdx.x == 0) {
        const unsigned long long k1 = passed + 1;
        const unsigned long long ngroups = (nblocks + kBarrierGroup - 1) / kBarrierGroup;
        const unsigned long long g = blockIdx.x / kBarrierGroup;
        const unsigned long long gsize = min((unsigned long long)kBarrierGroup, nblocks - g * kBarrierGroup);
        bool good = true;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        const unsigned long long old = atomicAdd(&sync->arrive[g].v, 1ull);
        if (old + 1 == k1 * gsize) {
            atomicAdd(&sync->top.v, 1ull);
            good = sync_wait(sync, &sync->top.v, k1 * ngroups);
            atomicAdd(&sync->release[g].v, 1ull);
        } else {
            good = sync_wait(sync, &sync->release[g].v, k1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        ok = good ? 1 : 0;
    }
    passed += 1;
    __syncthreads();
    return ok != 0;
}

// Occupancy floor of the persistent kernels: four workgroups per CU, five
// for int8 (whose march fits the registers of five without spilling, so its
// co-residency bound leaves room for a default grid of four per CU).
constexpr int persistent_min_blocks(int fmt) { return fmt == ISLF_SPIN_INT8 ? 5 : 4; }

template <int FMT>
__global__ __launch_bounds__(kBlock, persistent_min_blocks(FMT)) void k_persistent(const RepDesc *__restrict__ descs,
                                                       RepState *__restrict__ st,
                                                       const Entry *__restrict__ items,
                                                       const int *__restrict__ first,
                                                       const int *__restrict__ reps, int n_reps,
                                                       uint32_t n_sweeps, GridSync *sync)
{
    __shared__ Tables tb;
    const unsigned long long G = gridDim.x;
    const int b = plan_block();
    const int i0 = first[b], i1 = first[b + 1];
    unsigned long long passed = 0;
    int tb_key = -1;   // the workgroup's items are the same every stage: tables stay staged
    for (uint32_t s = 0; s < n_sweeps; ++s) {
        run_items<FMT, KIND_A, true>(descs, st, items, i0, i1, s, s ? FLAG_PREV : 0u, &tb, tb_key);
        if (!grid_barrier(sync, G, passed)) return;
        run_items<FMT, KIND_B, true>(descs, st, items, i0, i1, s, 0u, &tb, tb_key);
        // the record of sweep s-1 is complete since A(s); it is folded after
        // the workgroup's own B items (off the start of its stage), and before
        // the barrier that lets A(s+1) add to the same accumulator half
        if (s > 0) fold_waves<true>(descs, st, reps, n_reps, s - 1, 0u);
        if (!grid_barrier(sync, G, passed)) return;
    }
    run_items<FMT, KIND_F, true>(descs, st, items, i0, i1, n_sweeps - 1, 0u, &tb, tb_key);
    if (!grid_barrier(sync, G, passed)) return;
    fold_waves<true>(descs, st, reps, n_reps, n_sweeps - 1, n_sweeps);
}

// Barrier of one team (the workgroups of one replica): an arrival counter
// and a release counter on lines of their own; the last of the `size`
// members to arrive for barrier k bumps the release counter, which the
// members poll (the polls never touch the line the arrivals update).  The
// same ordering argument as grid_barrier (device-coherent accesses, every
// wave's memory operations complete before its workgroup arrives).
__device__ bool team_barrier(GridSync *sync, SyncLine *team, unsigned long long size, unsigned long long &passed)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    __shared__ int ok;
    if (threadIdx.x == 0) {
        const unsigned long long k1 = passed + 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        const unsigned long long old = atomicAdd(&team[0].v, 1ull);
        if (old + 1 == k1 * size) atomicAdd(&team[1].v, 1ull);
        const bool good = sync_wait(sync, &team[1].v, k1);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        ok = good ? 1 : 0;
    }
    passed += 1;
    __syncthreads();
    return ok != 0;
}

// The persistent schedule with team barriers: workgroup b runs its items
// (all of one replica) through the A / B launches of every sweep, meeting
// its team between them; rank 0 of a team folds its replica's records and,
// at the end, advances its sweep counter.  A barrier that gives up (bounded
// wait, or a raised error word) ends every workgroup at its next barrier.
template <int FMT>
__global__ __launch_bounds__(kBlock, persistent_min_blocks(FMT)) void k_persistent_teams(const RepDesc *__restrict__ descs,
                                                                RepState *__restrict__ st,
                                                                const Entry *__restrict__ items,
                                                                const int *__restrict__ first,
                                                                const TeamInfo *__restrict__ teams,
                                                                uint32_t n_sweeps, GridSync *sync,
                                                                SyncLine *rsync)
{
    __shared__ Tables tb;
    const int b = plan_block();
    const TeamInfo ti = teams[b];
    const int i0 = first[b], i1 = first[b + 1];
    SyncLine *ctr = rsync + 2 * ti.rep;   // arrival, release
    const unsigned long long size = (unsigned long long)ti.size;
    const bool folder = ti.rank == 0 && threadIdx.x < 64;   // wave 0 of rank 0
    const int lane = threadIdx.x & 63;
    unsigned long long passed = 0;
    int tb_key = -1;   // one replica per workgroup: its tables stay staged
    for (uint32_t s = 0; s < n_sweeps; ++s) {
        run_items<FMT, KIND_A, true>(descs, st, items, i0, i1, s, s ? FLAG_PREV : 0u, &tb, tb_key);
        if (!team_barrier(sync, ctr, size, passed)) return;
        run_items<FMT, KIND_B, true>(descs, st, items, i0, i1, s, 0u, &tb, tb_key);
        // sweep s-1's record, after the folder's own B items (see k_persistent)
        if (s > 0 && folder) fold_sweep<true>(descs[ti.rep], st[ti.rep], st[ti.rep].t + s - 1, lane);
        if (!team_barrier(sync, ctr, size, passed)) return;
    }
    run_items<FMT, KIND_F, true>(descs, st, items, i0, i1, n_sweeps - 1, 0u, &tb, tb_key);
    if (!team_barrier(sync, ctr, size, passed)) return;
    if (folder) {
        fold_sweep<true>(descs[ti.rep], st[ti.rep], st[ti.rep].t + n_sweeps - 1, lane);
        if (lane == 0) st[ti.rep].t += n_sweeps;
    }
}

// ---------------------------------------------------------------------------
// Initial states and format conversion.
// mode 0: random (Philox domain 1, t = 0; +1 iff the word's top bit is 0),
// mode 1: all up, 2: all down, 3: from staged host spins (int8 +-1, host layout).
// ---------------------------------------------------------------------------
__global__ void k_init_i8(const RepDesc *__restrict__ descs, int rep, int mode, const int8_t *__restrict__ host)
{
    const RepDesc &d = descs[rep];
    const int Lzh = d.Lz >> 1;
    // one 8-byte column (row, sublattice q, column k) per step: sites z = 2i + q, i = 8k .. 8k+7
    const long ncol = (long)d.Lx * d.Ly * 2 * d.K;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < ncol; c += (long)gridDim.x * blockDim.x) {
        const long row = c / (2 * d.K);
        const int rem = (int)(c - row * 2 * d.K);
        const int q = rem / d.K, k = rem - q * d.K;
        const int nv = min(8, Lzh - 8 * k);
        uint64_t W = 0;
        if (mode == 0) {
            for (int h = 0; h < 2; ++h) {
                uint32_t rnd[4];
                const uint32_t g = (((uint32_t)(row * d.C + 2 * k + h)) << 1) | (uint32_t)q;
                philox10(g, 0u, d.replica, 1u, d.key0, d.key1, rnd);
                for (int l = 0; l < 4; ++l) {
                    const int b = 4 * h + l;
                    if (b < nv) W |= (uint64_t)(1u - (rnd[l] >> 31)) << (8 * b);
                }
            }
        } else if (mode == 1) {
            for (int b = 0; b < nv; ++b) W |= 1ull << (8 * b);
        } else if (mode == 3) {
            const int8_t *src = host + row * d.Lz + q;
            for (int b = 0; b < nv; ++b) W |= (uint64_t)(src[2 * (8 * k + b)] > 0 ? 1u : 0u) << (8 * b);
        }
        *(uint64_t *)(d.spins + (size_t)row * d.RB + (size_t)q * d.Hp + 8 * k) = W;
    }
}

__global__ void k_init_bp(const RepDesc *__restrict__ descs, int rep, int mode, const int8_t *__restrict__ host)
{
    const RepDesc &d = descs[rep];
    const int nbits = d.Lz >> 1;
    const long nw = (long)d.Lx * d.Ly * 2 * d.Wq;
    uint32_t *words = (uint32_t *)d.spins;
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < nw; k += (long)gridDim.x * blockDim.x) {
        const long row = k / (2 * d.Wq);
        const int rem = (int)(k - row * 2 * d.Wq);
        const int q = rem / d.Wq, w = rem - q * d.Wq;
        const int nb_here = min(32, nbits - 32 * w);
        uint32_t S = 0;
        for (int b = 0; b < nb_here; ++b) {
            const int i = 32 * w + b;
            uint32_t u;
            if (mode == 0) {
                uint32_t rnd[4];
                const uint32_t g = (((uint32_t)(row * d.C + (i >> 2))) << 1) | (uint32_t)q;
                philox10(g, 0u, d.replica, 1u, d.key0, d.key1, rnd);
                u = 1u - (rnd[i & 3] >> 31);
            } else if (mode == 1) {
                u = 1;
            } else if (mode == 2) {
                u = 0;
            } else {
                u = host[row * d.Lz + 2 * i + q] > 0 ? 1u : 0u;
            }
            S |= u << b;
        }
        words[k] = S;
    }
}

// Internal format -> host layout int8 +-1.
__global__ void k_export(const RepDesc *__restrict__ descs, int rep, int8_t *__restrict__ out)
{
    const RepDesc &d = descs[rep];
    const int Lz = d.Lz;
    // a workgroup takes whole rows (x, y); the lanes run along z
    for (int r = blockIdx.x; r < d.Lx * d.Ly; r += gridDim.x) {
        int8_t *o = out + (size_t)r * (size_t)Lz;
        if (d.fmt == ISLF_SPIN_INT8) {
            const uint8_t *src = d.spins + (size_t)r * d.RB;
            for (int z = threadIdx.x; z < Lz; z += blockDim.x)
                o[z] = src[(z & 1) * d.Hp + (z >> 1)] ? (int8_t)1 : (int8_t)-1;
        } else {
            const uint32_t *row = (const uint32_t *)d.spins + (size_t)r * 2 * d.Wq;
            for (int z = threadIdx.x; z < Lz; z += blockDim.x)
                o[z] = bp_bit(row + (size_t)(z & 1) * d.Wq, z >> 1) ? (int8_t)1 : (int8_t)-1;
        }
    }
}

// ---------------------------------------------------------------------------
// Full recompute of (B, M, M1, Mn): each site counts its three forward slots.
// Works on the host-layout export so that it is one code for both formats.
// ---------------------------------------------------------------------------
__global__ void k_recompute(const RepDesc *__restrict__ descs, int rep, const int8_t *__restrict__ s,
                            unsigned long long *__restrict__ out)
{
    const RepDesc &d = descs[rep];
    const int Lx = d.Lx, Ly = d.Ly, Lz = d.Lz;
    const uint32_t plane = (uint32_t)Ly * (uint32_t)Lz;
    const int sg = d.seam_invert ? -1 : 1;
    // a workgroup takes whole rows (x, y), four at a time so that each lane
    // has the loads of four rows in flight: x and y are uniform, the lanes
    // run along z (coalesced), and offsets fit 32 bits (a replica is below
    // 4 GiB)
    int B = 0, M = 0, M1 = 0, Mn = 0;
    const int rows = Lx * Ly;
    for (int r0 = 4 * (int)blockIdx.x; r0 < rows; r0 += 4 * (int)gridDim.x) {
        // per row (uniform): offset, y-neighbour row offset and sign, x+1 plane
        uint32_t ro[4], yo[4];
        int ys[4], xp[4], ok[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int r = min(r0 + k, rows - 1);
            const int x = r / Ly, y = r - x * Ly;
            ok[k] = r0 + k < rows;
            ro[k] = (uint32_t)r * (uint32_t)Lz;
            yo[k] = y < Ly - 1 ? ro[k] + (uint32_t)Lz : (uint32_t)((d.seam_reflect ? Lx - 1 - x : x) * Ly) * Lz;
            ys[k] = y < Ly - 1 ? 1 : sg;
            xp[k] = x < Lx - 1;
        }
        int b[4] = {0, 0, 0, 0}, m[4] = {0, 0, 0, 0};
        for (int z = threadIdx.x; z < Lz; z += blockDim.x) {
            const int zn = z + 1 == Lz ? 0 : z + 1;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!ok[k]) break;
                const int si = s[ro[k] + z];
                int bb = si * s[ro[k] + zn] + ys[k] * si * s[yo[k] + z];
                if (xp[k]) bb += si * s[ro[k] + plane + z];
                b[k] += bb;
                m[k] += si;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!ok[k]) break;
            const int x = (r0 + k) / Ly;
            B += b[k];
            M += m[k];
            if (x == 0) M1 += m[k];
            if (x == Lx - 1) Mn += m[k];
        }
    }
    long long v[4] = {B, M, M1, Mn};
    __shared__ long long red[4][kBlock / 64];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        for (int k = 0; k < 4; ++k) red[k][threadIdx.x >> 6] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        long long acc = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) acc += red[threadIdx.x][w];
        atomicAdd(&out[threadIdx.x], (unsigned long long)acc);
    }
}

// Sets the running observables of a replica (after init / set_spins).
// Layer profile (Sec. II.B, Eq. 17): for every row (x, y) of replica rep,
// P = sum over z of its spins, written to out (int32) or, if out is NULL,
// added to acc (int64).  A workgroup owns R whole rows (R * words per row <=
// 1024 words, at least one row) and reads them as one coalesced run of 32-bit
// words (int8: four sites per word; bit-packed: 32 sites of one sublattice),
// masks the padding past Lz, and sums the up spins of each row in LDS;
// P = 2 * (up spins) - Lz.
constexpr int kProfileWords = 1024;
constexpr int kProfileRows = kProfileWords / 2;   // rows hold at least two words

__global__ __launch_bounds__(256) void k_layer_profile(const RepDesc *__restrict__ descs, int rep,
                                                       int32_t *__restrict__ out, long long *__restrict__ acc)
{
    __shared__ uint32_t cnt[kProfileRows];
    const RepDesc &d = descs[rep];
    const int Lz = d.Lz;
    const bool i8 = d.fmt == ISLF_SPIN_INT8;
    const uint32_t rw = i8 ? (uint32_t)(d.RB >> 2) : (uint32_t)(2 * d.Wq);   // words per row
    const long rows = (long)d.Lx * (long)d.Ly;
    const uint32_t R = rw >= (uint32_t)kProfileWords ? 1u : (uint32_t)kProfileWords / rw;
    const long r0 = (long)blockIdx.x * R;
    if (r0 >= rows) return;
    const uint32_t nr = (uint32_t)min((long)R, rows - r0);
    for (uint32_t k = threadIdx.x; k < nr; k += blockDim.x) cnt[k] = 0;
    __syncthreads();
    const gcu32 *base = (const gcu32 *)d.spins + (size_t)r0 * rw;
    const uint32_t nw = nr * rw;
    const int Wq = d.Wq, nbits = Lz >> 1;
    for (uint32_t k = threadIdx.x; k < nw; k += blockDim.x) {
        const uint32_t row = k / rw, col = k - row * rw;
        uint32_t v = base[k], up;
        if (i8) {
            // byte i0 .. i0+3 of sublattice row q; the padding past Lz/2 is masked
            const uint32_t hw = (uint32_t)d.Hp >> 2;
            const int i0 = 4 * (int)(col < hw ? col : col - hw);
            const int nb = min(4, (Lz >> 1) - i0);
            if (nb < 4) v &= nb <= 0 ? 0u : ((1u << (8 * nb)) - 1u);
            up = __builtin_amdgcn_sad_u8(v, 0u, 0u);
        } else {
            const int w = (int)col < Wq ? (int)col : (int)col - Wq;
            const int nb = min(32, nbits - 32 * w);
            if (nb < 32) v &= (1u << nb) - 1u;
            up = (uint32_t)__popc(v);
        }
        if (up) atomicAdd(&cnt[row], up);
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < nr; k += blockDim.x) {
        const int32_t P = 2 * (int32_t)cnt[k] - Lz;
        if (out) out[r0 + k] = P;
        else acc[r0 + k] += P;
    }
}

__global__ void k_set_state(RepState *st, int rep, const unsigned long long *obs, uint32_t t)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int k = 0; k < 4; ++k) st[rep].cur[k] = (long long)obs[k];
        st[rep].t = t;
        st[rep].live = 1;
    }
}

__global__ void k_zero_u64(unsigned long long *p, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Energies and means (Eq. 1, Eq. 19 integrand); thermodynamic integration.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double energy_of(double J, double H, double h1, double hn, double B, double M,
                                            double M1, double Mn)
{
    double e = -J * B;
    e = e - H * M;
    e = e - h1 * M1;
    e = e - hn * Mn;
    return e;
}

__global__ void k_energy(const islf_obs *__restrict__ rec, uint32_t cap, uint64_t first, uint32_t count,
                         double J, double H, double h1, double hn, double *__restrict__ out)
{
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x) {
        const islf_obs o = rec[(first + k) % cap];
        out[k] = energy_of(J, H, h1, hn, (double)o.B, (double)o.M, (double)o.M1, (double)o.Mn);
    }
}

// One block per replica: exact int64 sums of the records, then
// mean = (double)sum / (double)count; mean E from the means.
__global__ void k_means(const RepDesc *__restrict__ descs, const int *__restrict__ reps, uint64_t first, uint32_t count, double *__restrict__ out)
{
    const int i = blockIdx.x;
    const int r = reps[i];
    const RepDesc &d = descs[r];
    long long v[4] = {0, 0, 0, 0};
    for (uint32_t k = threadIdx.x; k < count; k += blockDim.x) {
        const islf_obs o = d.rec[(first + k) % d.cap];
        v[0] += o.B; v[1] += o.M; v[2] += o.M1; v[3] += o.Mn;
    }
    __shared__ long long red[4][kBlock / 64];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        for (int k = 0; k < 4; ++k) red[k][threadIdx.x >> 6] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m[4];
        for (int k = 0; k < 4; ++k) {
            long long s = 0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[k][w];
            m[k] = (double)s / (double)count;
        }
        out[5 * (size_t)i + 0] = energy_of(d.J, d.H, d.h1, d.hn, m[0], m[1], m[2], m[3]);
        for (int k = 0; k < 4; ++k) out[5 * (size_t)i + 1 + k] = m[k];
    }
}

__global__ void k_integrate(const double *__restrict__ h, const double *__restrict__ m1,
                            const double *__restrict__ mn, int n, double c1, double cn, double norm,
                            double *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double g_prev = norm * (c1 * m1[0] + cn * mn[0]);
    double acc = 0.0;
    out[0] = 0.0;
    for (int r = 1; r < n; ++r) {
        const double g = norm * (c1 * m1[r] + cn * mn[r]);
        const double step = 0.5 * (h[r] - h[r - 1]);
        acc = acc + step * (g_prev + g);
        out[r] = acc;
        g_prev = g;
    }
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free means (islf_means_noalloc): a file-scope
// device array of kNoAllocMaxReps x 5 doubles (320 KiB) that the means kernel
// writes in place of a staging buffer.  Each device holds its own copy for
// the life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns on that device, looked up once per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[5 * kNoAllocMaxReps];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_addr[kMaxDevices];

// The current device's address of `scratch` (looked up on its first use on
// that device, with that device current).
hipError_t noalloc_scratch(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[dev] = p;
    }
    *out = (double *)g_scratch_addr[dev];
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Host-callable launchers (used by islf_api.hip).
// ---------------------------------------------------------------------------
// kind 0 = A, 1 = B, 2 = F; grid = the plan's blocks (F: its slab blocks)
hipError_t launch_sweep(int fmt, int kind, const RepDesc *descs, RepState *st, const Entry *items,
                        const int *first, int grid, const int *reps, int n_reps, uint32_t s, uint32_t flags,
                        hipStream_t strm)
{
    if (grid <= 0) return hipSuccess;
    const dim3 g((unsigned int)grid), blk(kBlock);
    if (fmt == ISLF_SPIN_INT8) {
        if (kind == KIND_A)
            hipLaunchKernelGGL((k_sweep<ISLF_SPIN_INT8, KIND_A>), g, blk, 0, strm, descs, st, items, first, reps,
                               n_reps, s, flags);
        else if (kind == KIND_B)
            hipLaunchKernelGGL((k_sweep<ISLF_SPIN_INT8, KIND_B>), g, blk, 0, strm, descs, st, items, first, reps,
                               n_reps, s, flags);
        else
            hipLaunchKernelGGL((k_sweep<ISLF_SPIN_INT8, KIND_F>), g, blk, 0, strm, descs, st, items, first, reps,
                               n_reps, s, flags);
    } else {
        if (kind == KIND_A)
            hipLaunchKernelGGL((k_sweep<ISLF_SPIN_BITPACK, KIND_A>), g, blk, 0, strm, descs, st, items, first, reps,
                               n_reps, s, flags);
        else if (kind == KIND_B)
            hipLaunchKernelGGL((k_sweep<ISLF_SPIN_BITPACK, KIND_B>), g, blk, 0, strm, descs, st, items, first, reps,
                               n_reps, s, flags);
        else
            hipLaunchKernelGGL((k_sweep<ISLF_SPIN_BITPACK, KIND_F>), g, blk, 0, strm, descs, st, items, first, reps,
                               n_reps, s, flags);
    }
    return hipGetLastError();
}

// resident workgroups per CU of the A / B sweep kernels (the smaller)
hipError_t sweep_blocks_per_cu(int fmt, int *per_cu)
{
    int a = 0, b = 0;
    hipError_t e;
    if (fmt == ISLF_SPIN_INT8) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_sweep<ISLF_SPIN_INT8, KIND_A>, kBlock, 0);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_sweep<ISLF_SPIN_INT8, KIND_B>, kBlock, 0);
    } else {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_sweep<ISLF_SPIN_BITPACK, KIND_A>, kBlock, 0);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_sweep<ISLF_SPIN_BITPACK, KIND_B>, kBlock, 0);
    }
    *per_cu = e == hipSuccess ? (a < b ? a : b) : 0;
    return e;
}

hipError_t launch_fold(const RepDesc *descs, RepState *st, const int *reps, int n_reps, uint32_t s,
                       uint32_t advance, hipStream_t strm)
{
    if (n_reps <= 0) return hipSuccess;
    const int grid = (n_reps + kBlock / 64 - 1) / (kBlock / 64);
    hipLaunchKernelGGL(k_fold, dim3(grid), dim3(kBlock), 0, strm, descs, st, reps, n_reps, s, advance);
    return hipGetLastError();
}

const void *persistent_kernel(int fmt)
{
    return fmt == ISLF_SPIN_INT8 ? (const void *)k_persistent<ISLF_SPIN_INT8>
                                 : (const void *)k_persistent<ISLF_SPIN_BITPACK>;
}

hipError_t launch_persistent(int fmt, const RepDesc *descs, RepState *st, const Entry *items, const int *first,
                             const int *reps, int nreps, uint32_t nsweeps, GridSync *sync, int grid, hipStream_t s)
{
    void *args[] = {(void *)&descs, (void *)&st, (void *)&items, (void *)&first,
                    (void *)&reps, (void *)&nreps, (void *)&nsweeps, (void *)&sync};
    // fresh barrier counters for this launch (the error line is kept)
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, (unsigned long long *)&sync->top, 16L);
    hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, s, (unsigned long long *)&sync->arrive[0],
                       (long)(2 * kMaxGroups * 16));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipLaunchCooperativeKernel(persistent_kernel(fmt), dim3(grid), dim3(kBlock), args, 0, s);
}

const void *persistent_teams_kernel(int fmt)
{
    return fmt == ISLF_SPIN_INT8 ? (const void *)k_persistent_teams<ISLF_SPIN_INT8>
                                 : (const void *)k_persistent_teams<ISLF_SPIN_BITPACK>;
}

hipError_t launch_persistent_teams(int fmt, const RepDesc *descs, RepState *st, const Entry *items, const int *first,
                                   const TeamInfo *teams, uint32_t nsweeps, GridSync *sync, SyncLine *rsync,
                                   int n_rsync, int grid, hipStream_t s)
{
    void *args[] = {(void *)&descs, (void *)&st, (void *)&items, (void *)&first,
                    (void *)&teams, (void *)&nsweeps, (void *)&sync, (void *)&rsync};
    // fresh team counters for this launch (the error line is kept): two
    // lines per replica slot
    hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, s, (unsigned long long *)rsync, (long)n_rsync * 2 * 16);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipLaunchCooperativeKernel(persistent_teams_kernel(fmt), dim3(grid), dim3(kBlock), args, 0, s);
}

hipError_t launch_init(int fmt, const RepDesc *descs, int rep, int mode, const int8_t *host, hipStream_t s)
{
    if (fmt == ISLF_SPIN_INT8)
        hipLaunchKernelGGL(k_init_i8, dim3(1024), dim3(kBlock), 0, s, descs, rep, mode, host);
    else
        hipLaunchKernelGGL(k_init_bp, dim3(1024), dim3(kBlock), 0, s, descs, rep, mode, host);
    return hipGetLastError();
}

hipError_t launch_export(const RepDesc *descs, int rep, long rows, int8_t *out, hipStream_t s)
{
    const unsigned grid = (unsigned)std::max(1L, std::min(rows, 1L << 20));
    hipLaunchKernelGGL(k_export, dim3(grid), dim3(kBlock), 0, s, descs, rep, out);
    return hipGetLastError();
}

hipError_t launch_recompute(const RepDesc *descs, int rep, long rows, const int8_t *spins,
                            unsigned long long *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, out, 4L);
    // at most 1024 workgroups: each ends with four atomics on the same four
    // words, which serialise when there are many more
    const unsigned grid = (unsigned)std::max(1L, std::min((rows + 3) / 4, 1024L));
    hipLaunchKernelGGL(k_recompute, dim3(grid), dim3(kBlock), 0, s, descs, rep, spins, out);
    return hipGetLastError();
}

hipError_t launch_layer_profile(const RepDesc *descs, int rep, long rows, long words_per_row, int32_t *out,
                                long long *acc, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    // the kernel's rows per workgroup: kProfileWords / words per row, at least 1
    const long rw = words_per_row;
    const long R = rw >= kProfileWords ? 1 : kProfileWords / rw;
    const long grid = (rows + R - 1) / R;
    hipLaunchKernelGGL(k_layer_profile, dim3((unsigned int)grid), dim3(256), 0, s, descs, rep, out, acc);
    return hipGetLastError();
}

hipError_t launch_set_state(RepState *st, int rep, const unsigned long long *obs, uint32_t t, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_state, dim3(1), dim3(64), 0, s, st, rep, obs, t);
    return hipGetLastError();
}

hipError_t launch_zero(unsigned long long *p, long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3(256), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_energy(const islf_obs *rec, uint32_t cap, uint64_t first, uint32_t count, double J,
                         double H, double h1, double hn, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy, dim3(64), dim3(kBlock), 0, s, rec, cap, first, count, J, H, h1, hn, out);
    return hipGetLastError();
}

hipError_t launch_means(const RepDesc *descs, const int *reps, int n, uint64_t first, uint32_t count,
                        double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_means, dim3(n), dim3(kBlock), 0, s, descs, reps, first, count, out);
    return hipGetLastError();
}

hipError_t launch_integrate(const double *h, const double *m1, const double *mn, int n, double c1, double cn,
                            double norm, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_integrate, dim3(1), dim3(64), 0, s, h, m1, mn, n, c1, cn, norm, out);
    return hipGetLastError();
}

}  // namespace islf
