/*
 * islf — MI355X (gfx950) checkerboard Metropolis engine for the thin-film
 * nearest-neighbour Ising model of Block, Kim, Virnau and Binder,
 * "Anisotropic interfacial tension, contact angles, and line tensions: a
 * GPU-based Monte Carlo study of the Ising model" (arXiv:1411.5588).
 *
 * Plain C ABI: plain pointers and sizes, no C++ or framework types.  Every
 * entry point returns an islf_status; nothing throws across the boundary.
 * On failure islf_last_error() returns a thread-local message that stays valid
 * until the next call on the same thread.  Calls on one context are not
 * thread-safe; separate contexts are independent.
 *
 * Model (Sec. II.A, Eq. 1):
 *   E = -J sum_<ij> eps_ij S_i S_j - H sum_i S_i - h1 sum_{x=0} S_i - hn sum_{x=Lx-1} S_i
 * on an Lx x Ly x Lz simple-cubic film, S = +-1, periodic in z, free surfaces
 * at x = 0 (the paper's layer k_x = 1) and x = Lx-1 (layer k_x = n).  The y
 * boundary is periodic, antiperiodic, or the generalized antiperiodic
 * condition of Sec. II.A Eq. 11, S(k_x, k_y +- Ly, k_z) = -S(Lx+1-k_x, k_y, k_z):
 * the y-seam bond of site (x, Ly-1, z) joins (Lx-1-x, 0, z) with eps = -1.
 * Each site owns three forward bond slots (x+1 inside the film, z+1 mod Lz,
 * y+1 or the seam); a pair joined by two slots (Ly = 2 or Lz = 2) counts twice.
 *
 * Dynamics (Appendix: checkerboard update): one sweep runs four phases,
 * phase(x,y,z) = 2*[y == 0] + ((x+y+z) & 1), in the order 0,1,2,3; no bond
 * joins two sites of one phase under any of the three y boundaries, so every
 * site of a phase may be updated at once.  A site flips iff u < thr, where
 * u is a uint32 word of Philox4x32-10 (key = (seed mod 2^32, seed >> 32),
 * counter = (g, t, replica, 0), g = (((x*Ly+y)*ceil(Lz/8) + (z>>3)) << 1) | (z&1),
 * word (z>>1)&3, t = the replica's own sweep index) and
 * thr = 2^32 if dE <= 0 else floor(2^32 exp(-beta dE)), dE = 2 s (J n + h_site)
 * evaluated in IEEE double on the host once per parameter set.  A random
 * initial state uses counter (g, 0, replica, 1): spin +1 iff the top bit is 0.
 * Results are therefore a deterministic function of the inputs: the same
 * spins and observables for every execution form, tile shape and batch mix.
 *
 * Observables (Eq. 7 and the Eq. 19 integrand), one record per sweep:
 *   B  = sum over slots eps S_i S_j,  M = sum S,  M1 = sum_{x=0} S,  Mn = sum_{x=Lx-1} S.
 *
 * Host spin layout for set/get: int8 +-1 at s[(x*Ly + y)*Lz + z].
 */
#ifndef ISLF_H
#define ISLF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ISLF_OK = 0,
    ISLF_EINVAL = 1,   /* invalid argument or shape                          */
    ISLF_ENOMEM = 2,   /* device or host allocation failed                   */
    ISLF_EDEVICE = 3,  /* a HIP call failed                                  */
    ISLF_ESTATE = 4,   /* call not valid in the context's current state      */
    ISLF_ERANGE = 5    /* index out of range (Philox group, sweep, record)   */
} islf_status;

typedef enum { ISLF_YBC_PBC = 0, ISLF_YBC_APBC = 1, ISLF_YBC_GAPBC = 2 } islf_ybc;
typedef enum { ISLF_SPIN_INT8 = 0, ISLF_SPIN_BITPACK = 1 } islf_spin_format;
typedef enum { ISLF_INIT_RANDOM = 0, ISLF_INIT_UP = 1, ISLF_INIT_DOWN = 2, ISLF_INIT_HOST = 3 } islf_init;

/* How islf_sweep issues work.  All forms give bit-identical results.
 * A run of k sweeps is issued as launches A(0) B(0) A(1) B(1) ... B(k-1) F:
 * A(s) does phase 3 of sweep s-1 on row y = 0 (s > 0) and phase 0 of sweep
 * s, B(s) phases 1 and 2 of sweep s, F phase 3 of the last sweep, then a
 * small fold launch closes the run's last record.
 *  PLAIN      : the A and B launches go one replica at a time (one lattice
 *               per launch).
 *  BATCHED    : each A and B launch covers every replica of a concurrent
 *               replica group (islf_set_groups); the groups' launch chains
 *               run side by side on their own streams.
 *  PERSISTENT : one launch for all requested sweeps of every replica, with
 *               device-side grid barriers in place of the launch boundaries. */
typedef enum { ISLF_EXEC_PLAIN = 0, ISLF_EXEC_BATCHED = 1, ISLF_EXEC_PERSISTENT = 2 } islf_exec;

/* One replica (Sec. II.A Eq. 1 parameters plus the Markov-chain identity).
 * Lx >= 1, Ly >= 2, Lz >= 2 and even; beta in [0, +inf]; J, H, h1, hn finite.
 * h1 acts on x = 0, hn on x = Lx-1 (a one-layer film feels both, H + h1 + hn).
 * The paper's convention is hn = -h1 (Sec. II.A); any pair is accepted.  */
typedef struct {
    int32_t Lx, Ly, Lz;
    int32_t ybc;          /* islf_ybc                                       */
    double J, beta, H, h1, hn;
    uint64_t seed;        /* Philox key                                     */
    uint32_t replica;     /* enters the Philox counter; caller-chosen id    */
    int32_t init;         /* islf_init                                      */
} islf_replica_desc;

/* Observables after one completed sweep (exact integers). */
typedef struct {
    int64_t B, M, M1, Mn;
} islf_obs;

typedef struct islf_ctx islf_ctx;

/* Device allocator hooks (e.g. a framework's caching allocator).  alloc
 * returns a device pointer aligned to at least 256 bytes, or NULL. */
typedef void *(*islf_alloc_fn)(size_t bytes, void *user);
typedef void (*islf_free_fn)(void *ptr, void *user);

/* ---------------------------------------------------------------------- */
/* Context                                                                 */
/* ---------------------------------------------------------------------- */

/* Creates a context holding n_reps replicas (n_reps >= 1) in the given spin
 * format, each with a ring of obs_capacity (>= 3) per-sweep records, and
 * initialises every replica per its init field (ISLF_INIT_HOST starts all-up
 * until islf_set_spins is called).  hip_stream (hipStream_t, may be NULL for
 * the default stream) is borrowed: all device work of this context is ordered
 * on it (the batched form's group streams fork from it and join back to it
 * within each call).  Device memory comes from alloc/free if given, else hipMalloc.  On
 * failure nothing stays allocated and *out is NULL.
 * Errors: EINVAL (shape, n_reps, capacity, format), ERANGE (lattice too large
 * for the 32-bit Philox group counter), ENOMEM, EDEVICE. */
islf_status islf_create(const islf_replica_desc *reps, int32_t n_reps, int32_t spin_format,
                        uint32_t obs_capacity, void *hip_stream, islf_ctx **out);
islf_status islf_create_with_allocator(const islf_replica_desc *reps, int32_t n_reps,
                                       int32_t spin_format, uint32_t obs_capacity,
                                       void *hip_stream, islf_alloc_fn alloc,
                                       islf_free_fn free_fn, void *user, islf_ctx **out);

/* Synchronises the context's stream and releases everything it owns. */
islf_status islf_destroy(islf_ctx *ctx);

/* Number of replica slots, live or retired (slot indices run 0 .. n-1). */
islf_status islf_num_replicas(const islf_ctx *ctx, int32_t *n);

/* Copies a live replica's parameters as given at creation (ERANGE if the
 * slot is not live, so this also tells whether a slot holds a replica). */
islf_status islf_get_desc(const islf_ctx *ctx, int32_t rep, islf_replica_desc *out);

/* Host <-> device spins, int8 +-1 in the host layout above; n must equal
 * Lx*Ly*Lz.  set_spins also recomputes the initial observables and may only
 * be called before the replica's first sweep, or on a replica marked failed
 * by a persistent launch (see islf_sweep), which it restarts at sweep 0
 * (else ESTATE).  Both synchronise.
 * Errors: EINVAL (n, values other than +-1), ERANGE (rep), ESTATE. */
islf_status islf_set_spins(islf_ctx *ctx, int32_t rep, const int8_t *host, size_t n);
islf_status islf_get_spins(islf_ctx *ctx, int32_t rep, int8_t *host, size_t n);

/* ---------------------------------------------------------------------- */
/* Sweeps (Appendix: checkerboard update; Sec. II.A Eq. 1)                 */
/* ---------------------------------------------------------------------- */

/* Selects the execution form used by islf_sweep (islf_exec). */
islf_status islf_set_exec(islf_ctx *ctx, int32_t exec_mode);

/* Enqueues n_sweeps sweeps of every live replica on the context's stream and
 * returns without waiting.  Per sweep the per-flip changes of (B, M, M1, Mn)
 * are reduced inside the update kernels and one record is stored per replica.
 * Errors: ERANGE if a replica's sweep index would pass 2^32-1, EDEVICE,
 * ESTATE if a live replica is marked failed (below).
 *
 * Failure of a persistent launch: its grid barriers wait a bounded time; a
 * block that gives up raises an error word and every block of the launch
 * then stops at its next barrier, leaving the sweeps half done.  The next
 * call that reads results (measure, sweep_count, get_spins, recompute,
 * record_energy, means) returns EDEVICE and marks every live replica failed;
 * from then on calls on a failed replica (and sweeps, graph capture and
 * replay of a context holding one) return ESTATE until islf_set_spins
 * restarts it at sweep 0 or it is retired. */
islf_status islf_sweep(islf_ctx *ctx, uint32_t n_sweeps);

/* Sweep index of the replica = number of sweeps it has completed (synchronises). */
islf_status islf_sweep_count(islf_ctx *ctx, int32_t rep, uint64_t *t);

/* ---------------------------------------------------------------------- */
/* Measurement (Eq. 7, Eq. 19 integrands)                                  */
/* ---------------------------------------------------------------------- */

/* Copies records of sweeps first .. first+count-1 (0-based sweep numbers) of
 * one replica to host memory; synchronises.  The ring keeps the most recent
 * obs_capacity-1 records: older or not yet run sweeps give ERANGE. */
islf_status islf_measure(islf_ctx *ctx, int32_t rep, uint64_t first, uint32_t count, islf_obs *out);

/* Recomputes (B, M, M1, Mn) of the replica's current spins from scratch on
 * the device (a check of the fused per-sweep reductions); synchronises. */
islf_status islf_recompute(islf_ctx *ctx, int32_t rep, islf_obs *out);

/* Energies of one replica's records on the device: E = ((-J B - H M) - h1 M1)
 * - hn Mn (Eq. 1, IEEE double, left to right) of records first ..
 * first+count-1, computed by a kernel and copied to host out[count];
 * synchronises.  Errors as islf_measure. */
islf_status islf_record_energy(islf_ctx *ctx, int32_t rep, uint64_t first, uint32_t count, double *out);

/* Per-replica means over records first .. first+count-1 of every live
 * replica, computed on the device as (double)(exact int64 sum) / (double)count:
 * out[5*r + {0,1,2,3,4}] = mean {E, B, M, M1, Mn} (E by the islf_energy
 * formula, then averaged in index order).  Host out of 5*n_reps doubles;
 * synchronises.  Errors: ERANGE if a replica lacks a requested record. */
islf_status islf_means(islf_ctx *ctx, uint64_t first, uint32_t count, double *out);

/* The means of islf_means, with the same results and layout, for callers
 * that cannot allocate device memory (code between graph captures, tight
 * serving loops, harnesses that forbid allocation): no hipMalloc, hipFree or
 * allocator callback is called.  The kernel writes into a file-scope device
 * array of the library (5 doubles for each of at most 8192 live replicas,
 * 320 KiB, held on every device the library runs on until the process ends)
 * and the results are copied to the host; out holds 5 doubles per replica
 * slot (islf_num_replicas), NaN for retired slots.  The array is shared by
 * every call on one device: calls on contexts of the same device that
 * overlap in time (other threads) race, so serialise them.  Synchronises.
 * Errors: EINVAL (NULL), ERANGE (more than 8192 live replicas, or a replica
 * lacks a requested record), ESTATE (replica tables not current after
 * islf_set_tile, or a failed replica), EDEVICE. */
islf_status islf_means_noalloc(islf_ctx *ctx, uint64_t first, uint32_t count, double *out);

/* The same means for one replica: out[0..4] = mean {E, B, M, M1, Mn} over
 * its records first .. first+count-1.  Host out; synchronises. */
islf_status islf_replica_means(islf_ctx *ctx, int32_t rep, uint64_t first, uint32_t count, double *out);

/* ---------------------------------------------------------------------- */
/* Host FP64 post-processing (Sec. II.A Eq. 1, Eq. 9; Sec. II.C Eq. 22)    */
/* ---------------------------------------------------------------------- */

/* Energies of n observable records of one replica (Sec. II.A Eq. 1) on the
 * host in IEEE double, left to right, no fused multiply-add:
 *   E_out[k] = ((-J B_k - H M_k) - h1 M1_k) - hn Mn_k
 * with J, H, h1, hn taken from *desc (its other fields are not used).
 * desc, obs[n] and E_out[n] are host memory owned by the caller; no device
 * is touched and nothing is allocated.  n = 0 is a no-op.
 * Errors: EINVAL (NULL desc, or NULL obs / E_out with n > 0, or a
 * non-finite J, H, h1, hn). */
islf_status islf_energy(const islf_replica_desc *desc, const islf_obs *obs, size_t n, double *E_out);

/* Thermodynamic integration over the surface field (Eq. 9; Eq. 22 along the
 * field path of the inclined-interface film): a cumulative trapezoid on the
 * host in IEEE double, left to right, no fused multiply-add:
 *   g_r = norm * (c1 * mean_M1[r] + cn * mean_Mn[r]),  cumulative_out[0] = 0,
 *   cumulative_out[r] = cumulative_out[r-1] + (0.5 * (h[r] - h[r-1])) * (g_{r-1} + g_r).
 * (c1, cn) = (-1, -1) is the literal integrand of Eq. 9; (-1, +1) integrates
 * the field-conjugate -<m1 - mn> along hn = -h1 (the Eq. 7 derivative).  With
 * the means of the energy in place of mean_M1 / mean_Mn and (c1, cn) =
 * (1, -1) the same rule integrates U_a - U_b over beta (Eq. 19).  h, mean_M1,
 * mean_Mn and cumulative_out are host arrays of n doubles owned by the
 * caller (n >= 1); no device is touched and nothing is allocated.
 * Errors: EINVAL (n < 1, NULL). */
islf_status islf_integrate(const double *h, const double *mean_M1, const double *mean_Mn, int32_t n, double c1,
                           double cn, double norm, double *cumulative_out);

/* The same trapezoid run by a kernel: h, m1, mn, out are DEVICE pointers to
 * n doubles (n >= 1), enqueued on hip_stream without waiting, results
 * bit-identical to islf_integrate.  For a pipeline whose means already sit in
 * device memory.  Errors: EINVAL (n < 1, NULL), EDEVICE. */
islf_status islf_integrate_device(const double *h, const double *m1, const double *mn, int32_t n, double c1,
                                  double cn, double norm, double *out, void *hip_stream);

/* ---------------------------------------------------------------------- */
/* Batching and serving                                                    */
/* ---------------------------------------------------------------------- */

/* Device bytes one replica needs in a context (spins, ring, tables, work
 * lists), for admission by memory footprint. */
islf_status islf_footprint_bytes(const islf_replica_desc *desc, int32_t spin_format,
                                 uint32_t obs_capacity, uint64_t *bytes);

/* Admits a replica into a free slot (or a new one) of a running context and
 * initialises it; the replica starts at sweep 0 whatever the others' sweep
 * indices are, and its draws depend only on its own (seed, replica, t).
 * Synchronises.  Errors: EINVAL, ERANGE, ENOMEM. */
islf_status islf_batch_add(islf_ctx *ctx, const islf_replica_desc *desc, int32_t *slot);

/* Retires a replica: its slot stops sweeping and its device memory (spins,
 * records, accumulators) is released, so that the memory a context holds
 * follows its live replicas.  Synchronises.  Errors: ERANGE (slot not live). */
islf_status islf_batch_retire(islf_ctx *ctx, int32_t slot);

/* Device bytes the context holds now: *total over every allocation
 * (replica blocks, descriptor tables, launch plans, work lists, sync words),
 * *replica_bytes (optional) over the replicas' own blocks (spins, record
 * ring, accumulators), the part islf_footprint_bytes prices per replica.
 * Host only, no synchronisation.  Errors: EINVAL (NULL context or total). */
islf_status islf_device_bytes(const islf_ctx *ctx, uint64_t *total, uint64_t *replica_bytes);

/* Records k_sweeps sweeps of the current batch (in the current execution
 * form) as HIP graphs: one graph, or with concurrent replica groups
 * (islf_set_groups) one graph per group captured on the group's stream.
 * islf_run_graph replays them n_replays times, ordered after the work issued
 * before on the context's stream and before the work issued after it there
 * (the group streams fork from and join back to it).  Admitting or retiring
 * a replica, or changing the groups or the grid, invalidates the graphs
 * (run_graph then returns ESTATE until the next capture).  Errors: EINVAL,
 * ESTATE, EDEVICE. */
islf_status islf_graph_capture(islf_ctx *ctx, uint32_t k_sweeps);
islf_status islf_run_graph(islf_ctx *ctx, uint32_t n_replays);

/* ---------------------------------------------------------------------- */
/* Tuning                                                                  */
/* ---------------------------------------------------------------------- */

/* Number of tile variants of the update kernels, and the variant in use for
 * a replica.  Every variant computes the same result; they differ only in
 * the thread-to-site mapping.  islf_set_tile changes one replica's variant
 * (rebuilding work lists).
 * islf_autotune tunes the live batch in two steps; a trial is the shortest
 * of three timed runs of `sweeps` sweeps after one untimed run: (1) per size
 * class, every tile variant (the class's replicas alone, in a batched plan of
 * their own), the fastest kept if it beats the class's own variant by 1%;
 * (2) for the context's execution form, the launch configuration on the
 * whole batch: batched, concurrent groups 1..4 x workgroups per launch (1/2,
 * 1, 3/2 of the default) x share taper (0, 0.1, 0.2); persistent, grid or
 * team barriers x grids of up to one workgroup per CU below the co-residency
 * bound x tapers 0, 0.2, 0.4, 0.6.  The four fastest and the configuration in use
 * are timed again (shortest of six runs); a finalist replaces the one in use
 * only if it is 1% faster (islf_get_groups, islf_get_grid, islf_get_taper,
 * islf_get_barriers report the result).  Spins, records and sweep
 * counters are restored afterwards, so results are unaffected.  Synchronises.
 * Errors: EINVAL, ENOMEM (backups), EDEVICE. */
islf_status islf_num_tiles(int32_t spin_format, int32_t *n);
islf_status islf_get_tile(const islf_ctx *ctx, int32_t rep, int32_t *tile);
islf_status islf_set_tile(islf_ctx *ctx, int32_t rep, int32_t tile);
islf_status islf_autotune(islf_ctx *ctx, uint32_t sweeps);

/* Share taper of the batched and persistent launch plans: the work of a
 * launch is cut into per-workgroup shares that shrink linearly with the
 * dispatch rank by up to +-taper (later workgroups get less, against the
 * uneven progress of the workgroups resident on one CU).  A negative value
 * restores the built-in one (0 bit-packed and 0.1 int8 batched; 0.4
 * persistent, whose shares step down by dispatch round, one workgroup per CU
 * per round, since the workgroups resident on a CU progress oldest first).  Every choice computes the same result; changing it
 * invalidates a captured graph.  Errors: EINVAL (NULL, taper >= 1). */
islf_status islf_set_taper(islf_ctx *ctx, double taper);
islf_status islf_get_taper(const islf_ctx *ctx, double *taper);

/* Launch-plan preview, host only (no device, no context): the work items of
 * n_reps replicas (tile variant `tile`, or each replica's default with -1)
 * cut into the plan of one launch chain of `grid` workgroups, as the batched
 * form builds it.  For checking plans and choosing grids.
 *   shapes (optional, 4 x n_reps int32): per replica (tile variant, columns
 *     per box tile or 0 for a linear tile, rows per box tile, x planes per
 *     tile).
 *   items (optional, 6 x items_cap int32): per item (replica, x0, y0, j0,
 *     x steps, kind), kind 0 = main tile, 1 = seam-slab tile; a main tile's
 *     (y0, j0) is its first row and column (box) or its column range [y0, j0)
 *     over the plane's main rows 2 .. Ly-2 in row-major order (linear); a
 *     slab tile's x0, y0, j0, x steps are its first x pair, pairs, first
 *     column and columns.
 *   first (optional, first_cap int32): workgroup b runs items
 *     [first[b], first[b+1]); slab items sit in the first workgroups.
 * *n_items and *n_first receive the counts (query them with NULL buffers).
 * Errors: EINVAL (NULL count pointers, bad replica, format, tile or grid),
 * ERANGE (a buffer is smaller than its count; the counts are still set). */
islf_status islf_plan_preview(const islf_replica_desc *descs, int32_t n_reps, int32_t spin_format, int32_t tile,
                              int32_t grid, int32_t *shapes, int32_t *items, int32_t items_cap, int32_t *n_items,
                              int32_t *first, int32_t first_cap, int32_t *n_first);

/* Layer profile of one replica's current spins (Sec. II.B, Eq. 17): for
 * every row (x, y), P[x*Ly + y] = sum over z of S(x, y, z), i.e. Lz times the
 * paper's row magnetisation m_{k_x}(y).  islf_layer_profile writes P to
 * dev_out (device memory, Lx*Ly int32, caller-owned); islf_layer_profile_add
 * adds P to dev_acc (device memory, Lx*Ly int64, caller-owned) so that a
 * sampled average accumulates on the device.  Both are enqueued on the
 * context's stream after the work issued before them and do not
 * synchronise.  Errors: EINVAL (NULL pointer), ERANGE (replica not live),
 * EDEVICE. */
islf_status islf_layer_profile(islf_ctx *ctx, int32_t rep, int32_t *dev_out);
islf_status islf_layer_profile_add(islf_ctx *ctx, int32_t rep, int64_t *dev_acc);

/* Concurrent replica groups of the batched form.  The live replicas are dealt
 * into this many groups of about equal site counts; each group sweeps on its
 * own stream (group 0 on the context's stream, the others on streams the
 * context owns, forked from and joined back to the context's stream, also
 * inside a captured graph), so that the tail of one group's launch overlaps
 * the launches of the others.  Replicas are independent, so the results are
 * the same for every choice.  0 (the default) means min(3, live replicas);
 * 1 gives one launch chain over all replicas.  Changing it invalidates a
 * captured graph.  Errors: EINVAL (NULL context, groups < 0 or > 16). */
islf_status islf_set_groups(islf_ctx *ctx, int32_t groups);
islf_status islf_get_groups(const islf_ctx *ctx, int32_t *groups);

/* Workgroups per A / B launch of the batched and plain forms; the work of a
 * launch is split evenly over them.  0 (the default) means two per resident
 * slot of the sweep kernels on the device for one launch chain; concurrent
 * replica groups of the batched form together get 3/2 per slot, split
 * evenly (at least 64 per group); a nonzero value
 * applies to every group's launches.  For the persistent form it is the
 * grid of the cooperative launch, which must not exceed the co-residency
 * bound the library computes for the persistent kernel on the device (the
 * smaller of the runtime's occupancy and a count from the kernel's registers,
 * LDS and the CU's thread slots, times the CUs); its default is one
 * workgroup per CU below that bound.  islf_get_grid reports the count of one
 * launch of the context's form: of one group's launch with several groups;
 * for a persistent context, the grid of its cooperative launch.  Every choice
 * computes the same result.  Changing it invalidates a captured graph.
 * Errors: EINVAL (NULL context, workgroups < 0 or > 2^20), ERANGE (a
 * persistent context, or a persistent sweep, with a grid above the bound). */
islf_status islf_set_grid(islf_ctx *ctx, int32_t workgroups);
islf_status islf_get_grid(const islf_ctx *ctx, int32_t *workgroups);

/* Runs n_sweeps sweeps of every live replica in the batched form (no graph)
 * with HIP events around each launch on the context's stream, and returns
 * the mean duration in milliseconds and the launch count of each kind:
 * [0] A launches (phase 3 of the previous sweep on row 0, phase 0),
 * [1] B launches (phases 1 and 2), [2] the closing F + fold pair of the run.
 * The sweeps are real (they advance the chains).  Synchronises.
 * Errors: EINVAL, EDEVICE, ERANGE. */
islf_status islf_phase_timings(islf_ctx *ctx, uint32_t n_sweeps, double *mean_ms, uint32_t *launches);

/* Barriers of the persistent form.  ISLF_BARRIER_GRID: one plan over all
 * replicas and grid-wide barriers.  ISLF_BARRIER_TEAM: the
 * cooperative grid is dealt to the live replicas (one workgroup each, then
 * greedily to the replica with the most sites per workgroup), each
 * replica's work is split over its team of workgroups, and a team meets at a
 * barrier of its own between the launch stages, so replicas never wait for
 * each other (used when every live replica can have at least one workgroup,
 * else the grid form).  ISLF_BARRIER_AUTO (the default): team barriers for
 * int8 spins or batches of 8 or more replicas, grid barriers otherwise (the
 * faster form on the batches measured).  islf_autotune tries both.  All
 * compute the same result.
 * islf_get_barriers reports the form the next persistent launch uses (GRID
 * or TEAM).  Changing it invalidates a captured graph.  Errors: EINVAL. */
typedef enum { ISLF_BARRIER_GRID = 0, ISLF_BARRIER_TEAM = 1, ISLF_BARRIER_AUTO = 2 } islf_barrier_mode;
islf_status islf_set_barriers(islf_ctx *ctx, int32_t mode);
islf_status islf_get_barriers(const islf_ctx *ctx, int32_t *mode);

/* Thread-local message describing the last failure on this thread. */
const char *islf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ISLF_H */
