/*
 * Plain, slow CPU oracle for checkerboard Metropolis sweeps of the thin-film
 * nearest-neighbour Ising model (Block, Kim, Virnau, Binder, arXiv:1411.5588).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP implementation: the geometry is an explicit bond list,
 * every threshold is recomputed from the energy change at the moment it is
 * needed, and Philox4x32-10 is written out again here.
 *
 * What it computes (section/equation of the paper in brackets):
 *  - Hamiltonian (Sec. II.A, Eq. 1): H = -J sum_<ij> S_i S_j - H sum_i S_i
 *    - H1 sum_{i in layer 1} S_i - Hn sum_{i in layer n} S_i, S_i = +-1.
 *  - Geometry (Sec. II.A, Fig. 1): Lx x Ly x Lz, periodic in z, two free
 *    surfaces x = 0 (paper layer k_x = 1, field h1) and x = Lx-1 (layer
 *    k_x = n = Lx, field hn).
 *  - y boundary (Sec. II.A, Eq. 11): PBC, APBC, or the generalized
 *    antiperiodic condition S(k_x,k_y,k_z) = -S(Lx+1-k_x, k_y +- Ly, k_z),
 *    i.e. 0-based x -> Lx-1-x with a sign change across the y seam.
 *  - Update: checkerboard single-spin-flip Metropolis (Appendix), acceptance
 *    min(1, exp(-beta dE)) realised as  u < thr  with u a uint32 Philox word
 *    and thr = 2^32 if dE <= 0 else floor(2^32 exp(-beta dE)).
 *  - Observables (Eq. 7 and Eq. 19 integrands): bond sum B, magnetisation M,
 *    surface-layer sums M1 (x = 0) and Mn (x = Lx-1), recomputed in full.
 *  - Layer profile (Eq. 17): the sum over z of the spins of every (x, y) row.
 *  - Thermodynamic integration over the surface field (Eq. 9, Eq. 22) by the
 *    trapezoid rule.
 *
 * Readings where the paper is silent (the full list is kept with the design
 * notes): 0-based coordinates, x = 0 is layer k_x = 1; each site owns three
 * forward bond slots (x+1 if x < Lx-1, z+1 mod Lz, y+1 or the seam), and a
 * pair linked through two slots (Ly = 2 or Lz = 2) carries 2J; phase of a site
 * = 2*[y == 0] + ((x+y+z) & 1), phases run 0,1,2,3 once per sweep (a two-colour
 * checkerboard is not a valid schedule under the generalized antiperiodic
 * condition when Lx+Ly is even); draws come from Philox4x32-10 with key
 * (seed mod 2^32, seed >> 32) and counter (g, t, replica, domain) where
 * g = (((x*Ly + y) * ceil(Lz/8) + (z >> 3)) << 1) | (z & 1) and the word used
 * is lane (z >> 1) & 3; domain 0 = sweeps (t = the replica's sweep index),
 * domain 1 = random initial state (t = 0, spin +1 iff the word's top bit is 0).
 *
 * Spin layout shared with callers: s[(x*Ly + y)*Lz + z] = +1 or -1 (int8).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PBC 0
#define OR_APBC 1
#define OR_GAPBC 2
#define OR_MAXNB 6

typedef struct {
    int32_t Lx, Ly, Lz, ybc;
    double J, beta, H, h1, hn;
    uint64_t seed;
    uint32_t replica;
    int64_t N;
    int32_t *nbr;   /* N * OR_MAXNB neighbour site indices          */
    int8_t *eps;    /* N * OR_MAXNB bond signs (+1, or -1 on a seam) */
    int8_t *nnb;    /* N neighbour counts                            */
    uint8_t *phase; /* N checkerboard phases 0..3                    */
    int32_t *fwd;   /* N * 3 forward slot targets (-1: no slot)      */
    int8_t *fwd_eps;/* N * 3 forward slot signs                      */
} or_lattice;

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random  */
/* numbers: as easy as 1, 2, 3").  Ten rounds of a multiply-hi/lo S-box */
/* on a 4-word counter; the 2-word key is bumped by the Weyl constants  */
/* between rounds.                                                      */
/* ------------------------------------------------------------------ */
static void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t mult_a = 0xD2511F53u, mult_b = 0xCD9E8D57u;
    const uint32_t weyl_a = 0x9E3779B9u, weyl_b = 0xBB67AE85u;
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k[2] = {key_in[0], key_in[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k[0] += weyl_a;
            k[1] += weyl_b;
        }
        uint64_t pa = (uint64_t)mult_a * (uint64_t)c[0];
        uint64_t pb = (uint64_t)mult_b * (uint64_t)c[2];
        uint32_t a_hi = (uint32_t)(pa >> 32), a_lo = (uint32_t)pa;
        uint32_t b_hi = (uint32_t)(pb >> 32), b_lo = (uint32_t)pb;
        uint32_t n0 = b_hi ^ c[1] ^ k[0];
        uint32_t n1 = b_lo;
        uint32_t n2 = a_hi ^ c[3] ^ k[1];
        uint32_t n3 = a_lo;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

void oracle_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    or_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------ */
/* Geometry: coordinates, forward bond slots, neighbour lists, phases. */
/* ------------------------------------------------------------------ */
static int64_t or_site(const or_lattice *L, int64_t x, int64_t y, int64_t z)
{
    return (x * L->Ly + y) * L->Lz + z;
}

static void or_coords(const or_lattice *L, int64_t i, int64_t *x, int64_t *y, int64_t *z)
{
    *z = i % L->Lz;
    *y = (i / L->Lz) % L->Ly;
    *x = i / ((int64_t)L->Lz * L->Ly);
}

/* Destination and sign of the y-forward slot leaving row y = Ly-1
 * (Sec. II.A: PBC, APBC, and Eq. 11 for the generalized condition). */
static void or_seam(const or_lattice *L, int64_t x, int64_t *x_to, int *sign)
{
    switch (L->ybc) {
    case OR_PBC:  *x_to = x;              *sign = +1; break;
    case OR_APBC: *x_to = x;              *sign = -1; break;
    default:      *x_to = L->Lx - 1 - x;  *sign = -1; break;
    }
}

static void or_add_nb(or_lattice *L, int64_t i, int64_t j, int sign)
{
    int k = L->nnb[i];
    L->nbr[i * OR_MAXNB + k] = (int32_t)j;
    L->eps[i * OR_MAXNB + k] = (int8_t)sign;
    L->nnb[i] = (int8_t)(k + 1);
}

void oracle_free(or_lattice *L)
{
    if (!L) return;
    free(L->nbr); free(L->eps); free(L->nnb); free(L->phase);
    free(L->fwd); free(L->fwd_eps);
    free(L);
}

/* Returns NULL on invalid parameters (Lx < 1, Ly < 2, Lz < 2 or odd). */
or_lattice *oracle_new(int32_t Lx, int32_t Ly, int32_t Lz, int32_t ybc,
                       double J, double beta, double H, double h1, double hn,
                       uint64_t seed, uint32_t replica)
{
    if (Lx < 1 || Ly < 2 || Lz < 2 || (Lz & 1) || ybc < 0 || ybc > 2) return NULL;
    or_lattice *L = (or_lattice *)calloc(1, sizeof(or_lattice));
    if (!L) return NULL;
    L->Lx = Lx; L->Ly = Ly; L->Lz = Lz; L->ybc = ybc;
    L->J = J; L->beta = beta; L->H = H; L->h1 = h1; L->hn = hn;
    L->seed = seed; L->replica = replica;
    L->N = (int64_t)Lx * Ly * Lz;
    L->nbr = (int32_t *)malloc(sizeof(int32_t) * L->N * OR_MAXNB);
    L->eps = (int8_t *)malloc(sizeof(int8_t) * L->N * OR_MAXNB);
    L->nnb = (int8_t *)calloc(L->N, 1);
    L->phase = (uint8_t *)malloc(L->N);
    L->fwd = (int32_t *)malloc(sizeof(int32_t) * L->N * 3);
    L->fwd_eps = (int8_t *)malloc(L->N * 3);
    if (!L->nbr || !L->eps || !L->nnb || !L->phase || !L->fwd || !L->fwd_eps) {
        oracle_free(L);
        return NULL;
    }
    for (int64_t i = 0; i < L->N; ++i) {
        int64_t x, y, z;
        or_coords(L, i, &x, &y, &z);
        /* slot 0: +x, only inside the film (free surfaces at x = 0, Lx-1) */
        if (x < Lx - 1) {
            L->fwd[3 * i + 0] = (int32_t)or_site(L, x + 1, y, z);
            L->fwd_eps[3 * i + 0] = +1;
        } else {
            L->fwd[3 * i + 0] = -1;
            L->fwd_eps[3 * i + 0] = 0;
        }
        /* slot 1: +z, periodic */
        L->fwd[3 * i + 1] = (int32_t)or_site(L, x, y, (z + 1) % Lz);
        L->fwd_eps[3 * i + 1] = +1;
        /* slot 2: +y, or across the seam */
        if (y < Ly - 1) {
            L->fwd[3 * i + 2] = (int32_t)or_site(L, x, y + 1, z);
            L->fwd_eps[3 * i + 2] = +1;
        } else {
            int64_t xt; int sg;
            or_seam(L, x, &xt, &sg);
            L->fwd[3 * i + 2] = (int32_t)or_site(L, xt, 0, z);
            L->fwd_eps[3 * i + 2] = (int8_t)sg;
        }
        L->phase[i] = (uint8_t)(2 * (y == 0) + ((x + y + z) & 1));
    }
    /* neighbour lists: every slot is seen from both of its ends */
    for (int64_t i = 0; i < L->N; ++i) {
        for (int k = 0; k < 3; ++k) {
            int64_t j = L->fwd[3 * i + k];
            if (j < 0) continue;
            or_add_nb(L, i, j, L->fwd_eps[3 * i + k]);
            or_add_nb(L, j, i, L->fwd_eps[3 * i + k]);
        }
    }
    return L;
}

int64_t oracle_nsites(const or_lattice *L) { return L->N; }

int32_t oracle_neighbours(const or_lattice *L, int64_t i, int32_t *nb, int8_t *sg)
{
    int k = L->nnb[i];
    for (int q = 0; q < k; ++q) {
        nb[q] = L->nbr[i * OR_MAXNB + q];
        sg[q] = L->eps[i * OR_MAXNB + q];
    }
    return k;
}

int32_t oracle_phase(const or_lattice *L, int64_t i) { return L->phase[i]; }

/* ------------------------------------------------------------------ */
/* Metropolis acceptance                                               */
/* ------------------------------------------------------------------ */

/* Field felt by a site of layer x (Eq. 1): bulk H, plus h1 on x = 0 and hn on
 * x = Lx-1; a one-layer film carries both, added in that order. */
static double or_site_field(const or_lattice *L, int64_t x)
{
    double h = L->H;
    if (x == 0) h = h + L->h1;
    if (x == L->Lx - 1) h = h + L->hn;
    return h;
}

static int64_t or_local_sum(const or_lattice *L, const int8_t *s, int64_t i)
{
    int64_t n = 0;
    for (int q = 0; q < L->nnb[i]; ++q)
        n += (int64_t)L->eps[i * OR_MAXNB + q] * s[L->nbr[i * OR_MAXNB + q]];
    return n;
}

/* Energy change of flipping site i: dE = 2 s_i (J n_i + h_i). */
double oracle_delta_e(const or_lattice *L, const int8_t *s, int64_t i)
{
    int64_t x, y, z;
    or_coords(L, i, &x, &y, &z);
    double n = (double)or_local_sum(L, s, i);
    double h = or_site_field(L, x);
    return 2.0 * (double)s[i] * (L->J * n + h);
}

/* Acceptance threshold on the uint32 draw: accept iff u < thr. */
uint64_t oracle_threshold_of_de(double beta, double dE)
{
    if (dE <= 0.0) return (uint64_t)1 << 32;
    double p = exp(-(beta * dE));
    return (uint64_t)floor(ldexp(p, 32));
}

uint64_t oracle_site_threshold(const or_lattice *L, const int8_t *s, int64_t i)
{
    return oracle_threshold_of_de(L->beta, oracle_delta_e(L, s, i));
}

/* The uint32 word drawn for site i in sweep t (domain 0) or at init (domain 1). */
uint32_t oracle_site_draw(const or_lattice *L, int64_t i, uint32_t t, uint32_t domain)
{
    int64_t x, y, z;
    or_coords(L, i, &x, &y, &z);
    int64_t chunks = (L->Lz + 7) / 8;
    uint64_t g = ((uint64_t)((x * L->Ly + y) * chunks + (z >> 3)) << 1) | (uint64_t)(z & 1);
    uint32_t lane = (uint32_t)((z >> 1) & 3);
    uint32_t ctr[4] = {(uint32_t)g, t, L->replica, domain};
    uint32_t key[2] = {(uint32_t)(L->seed & 0xFFFFFFFFu), (uint32_t)(L->seed >> 32)};
    uint32_t out[4];
    or_philox4x32_10(ctr, key, out);
    return out[lane];
}

/* Largest group index a lattice needs must fit the 32-bit counter word. */
int32_t oracle_counter_fits(const or_lattice *L)
{
    int64_t chunks = (L->Lz + 7) / 8;
    int64_t gmax = ((((int64_t)L->Lx * L->Ly) * chunks) << 1);
    return gmax <= ((int64_t)1 << 32);
}

/* init: 0 = random (Philox domain 1), 1 = all up, 2 = all down */
void oracle_init(const or_lattice *L, int8_t *s, int32_t init)
{
    for (int64_t i = 0; i < L->N; ++i) {
        if (init == 1) s[i] = +1;
        else if (init == 2) s[i] = -1;
        else s[i] = (oracle_site_draw(L, i, 0, 1) >> 31) ? -1 : +1;
    }
}

static void or_visit(const or_lattice *L, int8_t *s, int64_t i, uint32_t t)
{
    uint64_t thr = oracle_site_threshold(L, s, i);
    uint32_t u = oracle_site_draw(L, i, t, 0);
    if ((uint64_t)u < thr) s[i] = (int8_t)(-s[i]);
}

/* One sweep with sweep index t: phases 0, 1, 2, 3 in order, every site of a
 * phase visited once.  If order != NULL the sites of each phase are visited in
 * the order order[0..N) (a permutation), which must not change the result. */
void oracle_sweep(const or_lattice *L, int8_t *s, uint32_t t, const int64_t *order)
{
    for (int p = 0; p < 4; ++p) {
        for (int64_t k = 0; k < L->N; ++k) {
            int64_t i = order ? order[k] : k;
            if (L->phase[i] == p) or_visit(L, s, i, t);
        }
    }
}

/* Apply a single phase p of sweep t (used by the detailed-balance tests). */
void oracle_phase_step(const or_lattice *L, int8_t *s, uint32_t t, int32_t p)
{
    for (int64_t i = 0; i < L->N; ++i)
        if (L->phase[i] == p) or_visit(L, s, i, t);
}

/* Full recompute of B = sum over slots eps s_i s_j, M, M1 (x = 0), Mn (x = Lx-1). */
void oracle_observables(const or_lattice *L, const int8_t *s, int64_t out[4])
{
    int64_t B = 0, M = 0, M1 = 0, Mn = 0;
    for (int64_t i = 0; i < L->N; ++i) {
        int64_t x, y, z;
        or_coords(L, i, &x, &y, &z);
        for (int k = 0; k < 3; ++k) {
            int64_t j = L->fwd[3 * i + k];
            if (j >= 0) B += (int64_t)L->fwd_eps[3 * i + k] * s[i] * s[j];
        }
        M += s[i];
        if (x == 0) M1 += s[i];
        if (x == L->Lx - 1) Mn += s[i];
    }
    out[0] = B; out[1] = M; out[2] = M1; out[3] = Mn;
}

/* Layer profile (Sec. II.B, Eq. 17): out[x*Ly + y] = sum over z of S(x, y, z),
 * i.e. Lz times the paper's row magnetisation m_{k_x}(y). */
void oracle_layer_profile(const or_lattice *L, const int8_t *s, int64_t *out)
{
    for (int64_t r = 0; r < (int64_t)L->Lx * L->Ly; ++r) out[r] = 0;
    for (int64_t i = 0; i < L->N; ++i) {
        int64_t x, y, z;
        or_coords(L, i, &x, &y, &z);
        out[x * L->Ly + y] += s[i];
    }
}

/* E = -J B - H M - h1 M1 - hn Mn (Eq. 1), evaluated left to right in FP64,
 * at observables given as doubles: an exact record, or the means of records
 * (the energy is linear in them, so the mean energy is E at the means). */
double oracle_energy_at(double J, double H, double h1, double hn, const double obs[4])
{
    double e = -J * obs[0];
    e = e - H * obs[1];
    e = e - h1 * obs[2];
    e = e - hn * obs[3];
    return e;
}

/* The same for one integer record (B, M, M1, Mn). */
double oracle_energy(double J, double H, double h1, double hn, const int64_t obs[4])
{
    const double d[4] = {(double)obs[0], (double)obs[1], (double)obs[2], (double)obs[3]};
    return oracle_energy_at(J, H, h1, hn, d);
}

/* Run sweeps t0 .. t0+n-1, recording (B, M, M1, Mn) after each one. */
void oracle_run(const or_lattice *L, int8_t *s, uint32_t t0, uint32_t n, int64_t *records)
{
    for (uint32_t k = 0; k < n; ++k) {
        oracle_sweep(L, s, t0 + k, NULL);
        oracle_observables(L, s, records + 4 * (int64_t)k);
    }
}

/* Mean of count integer records: (double)sum / (double)count. */
double oracle_mean(const int64_t *values, int64_t stride, int64_t count)
{
    int64_t acc = 0;
    for (int64_t k = 0; k < count; ++k) acc += values[k * stride];
    return (double)acc / (double)count;
}

/* Thermodynamic integration over the surface field (Eq. 9 / Eq. 22):
 * g_r = norm (c1 m1_r + cn mn_r); I_0 = 0,
 * I_{r+1} = I_r + 0.5 (h_{r+1} - h_r)(g_r + g_{r+1}). */
void oracle_integrate(const double *h, const double *m1, const double *mn, int32_t n,
                      double c1, double cn, double norm, double *cum)
{
    if (n <= 0) return;
    double g_prev = norm * (c1 * m1[0] + cn * mn[0]);
    cum[0] = 0.0;
    for (int32_t r = 1; r < n; ++r) {
        double g = norm * (c1 * m1[r] + cn * mn[r]);
        double step = 0.5 * (h[r] - h[r - 1]);
        cum[r] = cum[r - 1] + step * (g_prev + g);
        g_prev = g;
    }
}
