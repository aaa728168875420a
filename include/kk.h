/*
 * kk.h -- C ABI of libkk: Metropolis-Kawasaki exchange sweeps of a binary
 * lipid mixture on a periodic square lattice, run on one AMD Instinct
 * MI355X (gfx950) with hand-written HIP kernels.
 *
 * The method is the one of Lis & Pintal, "GPU-Based Massive Parallel
 * Kawasaki Kinetics in Monte Carlo Modelling of Lipid Microdomains":
 *  - lipids of type A (0) and B (1) fill the lattice; a move exchanges two
 *    nearest neighbours (Kawasaki kinetics), so the composition never changes
 *    (Materials and Methods, "Monte Carlo model with Kawasaki based kinetics");
 *  - the only parameter is omega_AB = g_AB - (g_AA + g_BB)/2 in units of kT,
 *    and a move that changes the number of unlike contacts N_AB by dU is
 *    accepted with the Metropolis probability min(1, exp(-omega * dU))
 *    (same section, the Metropolis criterion and the omega_AB equation);
 *  - a sweep ("step") decomposes the lattice into disjoint domains many times
 *    and lets every domain centre try one exchange at once, N attempts per
 *    sweep in total (section "Massive Parallel Kawasaki Kinetics");
 *  - cluster sizes of one species are the analysed observable (section
 *    "Cluster Analysis methods").
 * The square-lattice decomposition (8 conflict-free centre classes in a
 * random order per sweep), the Philox4x32-10 random-number layout and the
 * 42-bit acceptance threshold make every result bit-reproducible and
 * independent of how the GPU tiles the lattice.
 *
 * Conventions for every call:
 *  - Lattices cross the boundary as host arrays of L*L bytes, row-major
 *    (index y*L + x), each 0 or 1.  The caller owns every host buffer; the
 *    library never keeps a pointer to one after the call returns.
 *  - A kk_sim owns all of its device memory and (unless one is supplied) its
 *    own HIP stream on the device that was current at creation.
 *  - Calls block until their GPU work is done, except kk_sweep_async.
 *  - A handle is not thread-safe: use one handle per thread.
 *  - Errors return a kk_status; kk_last_error() gives this thread's message.
 *    After KK_EDEVICE the handle is poisoned and later calls return
 *    KK_ESTATE (destroy it).
 */
#ifndef KK_H
#define KK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kk_sim kk_sim;

typedef enum {
    KK_OK = 0,
    KK_EINVAL = 1,  /* bad argument (NULL, out of range, wrong size) */
    KK_ENOMEM = 2,  /* device or host allocation failed */
    KK_EDEVICE = 3, /* a HIP call failed; the handle is poisoned */
    KK_ESTATE = 4,  /* the handle was poisoned by an earlier device error */
    KK_ETRUNC = 5   /* output capacity too small; *n_out holds the size needed */
} kk_status;

enum {
    KK_LAYOUT_AUTO = 0,     /* bit-packed when L % 32 == 0, else int8 */
    KK_LAYOUT_INT8 = 1,     /* device lattice: one byte (0/1) per site */
    KK_LAYOUT_BITPACKED = 2 /* device lattice: one bit per site, L/32 uint32 per row; needs L % 32 == 0 */
};

typedef struct {
    uint64_t size;  /* cluster size in sites */
    uint64_t count; /* number of clusters of that size */
} kk_hist_entry;

/* Create a simulation: an L x L periodic lattice with n1 = floor(composition*L*L + 0.5)
 * sites of type 1 placed uniformly at random from `seed` (the paper's random start,
 * Results, "MPKK vs. Kawasaki method"), interaction omega_kT (any finite value;
 * positive favours demixing), sweep counter t = 0.
 * L must be a multiple of 4 in [4, 32768] (a multiple of 32 for the bit-packed layout);
 * composition must lie in [0, 1].  *out receives the handle (NULL on failure). */
kk_status kk_create(kk_sim **out, uint32_t L, double composition, double omega_kT, uint64_t seed);

/* kk_create with an explicit device layout (KK_LAYOUT_*) and an optional HIP
 * stream (hipStream_t passed as void*; NULL = the handle creates its own).
 * A supplied stream must outlive the handle. */
kk_status kk_create_ex(kk_sim **out, uint32_t L, double composition, double omega_kT, uint64_t seed,
                       uint32_t layout, void *hip_stream);

/* Create a simulation on the paper's own lattice (Materials and Methods, Fig. 2
 * and "Cluster Analysis methods"): triangular, six neighbours, helical
 * boundaries.  Sites i = y*L + x (0 <= i < N = L*L) form one ring; the
 * neighbours of i are i +- 1, i +- L and i +- (L-1) mod N, so N_AB counts the
 * 3N bonds (i, i+1), (i, i+L), (i, i+L-1).  L must satisfy L % 8 == 4,
 * 4 <= L <= 32764; the lattice is stored one byte per site (KK_LAYOUT_INT8) and
 * initialised exactly as kk_create's random start.  A sweep is N attempts in 16
 * conflict-free classes (class(i) = i mod 16), run in a random order:
 *   class order of sweep t: Philox words of blocks (j, 0, t_lo, t_hi28 | 7<<28),
 *     j = 0..3, w[0..15]; Fisher-Yates from the identity, step k = 15..1 swaps
 *     entries k and (w[15-k] * (k+1)) >> 32;
 *   site i at sweep t: block (i/2, 0, t_lo, t_hi28 | 6<<28); word 2(i%2) picks
 *     the partner direction d = (w * 6) >> 32 (offsets +1, -1, +L, -L, +(L-1),
 *     -(L-1)), word 2(i%2)+1 is the uniform U;
 *   unlike pair (i, b) with n unlike neighbours (each excluding the other,
 *     0..10): exchange iff U < T[n] = min(2^32, ceil(exp(-omega (10-2n)) 2^32)).
 * kk_sweep, kk_sweep_async, kk_sweep_timed (16 launches per sweep), kk_energy,
 * kk_cluster_hist (six-connected clusters), kk_observe and kk_sweep_series
 * (similar_exact = 1 - N_AB/(3N); similar_sampled draws one of the six
 * neighbours with d = (w*6)>>32 from word i%4 of block (i/4, 1, t_lo,
 * t_hi28 | 5<<28)), kk_get_lattice, kk_set_lattice, kk_stats, kk_info and
 * kk_stream work on it; kk_thresholds, kk_set_tile, kk_get_tile and
 * kk_autotune return KK_EINVAL. */
kk_status kk_create_triangular(kk_sim **out, uint32_t L, double composition, double omega_kT, uint64_t seed,
                               void *hip_stream);

/* Triangular schemes for kk_create_triangular_ex. */
enum {
    KK_TRI_CLASSES = 0, /* the conflict-free 16-class schedule of kk_create_triangular */
    KK_TRI_MPKK = 1     /* the paper's literal MPKK (Materials and Methods, "Massive Parallel Kawasaki
                           Kinetics", Fig. 4), a comparison variant */
};

/* A triangular helical lattice of H rows of L sites (N = L*H, i = y*L + x on
 * one ring; neighbours i +- 1, i +- L, i +- (L-1) mod N), int8, placed as
 * kk_create's random start (Philox init keys addressed by (y, x)).
 * KK_TRI_CLASSES: as kk_create_triangular; needs L % 8 == 4 and H % 4 == 0.
 * KK_TRI_MPKK: needs L % 7 in {3, 5} and H % 7 == 0, so that the 7-site domains
 *   (a centre and its six neighbours) centred on c = k (mod 7) partition the
 *   ring for every k.  One "sweep" is one MPKK step of 7 iterations; iteration
 *   j draws k_j = (w * 7) >> 32 from word j%4 of Philox block (j/4, 2, t_lo,
 *   t_hi28 | 8<<28), with replacement, and makes one attempt in every domain
 *   m (centre k_j + 7m): direction d = (w * 6) >> 32 from word 2(m%2) and U
 *   from word 2(m%2)+1 of block (m/2, j, t_lo, t_hi28 | 9<<28), accepted iff
 *   U < T[n] as above.  All domains of an iteration decide from the lattice as
 *   it stood when the iteration began and their exchanges are applied
 *   together (the domains are disjoint): the paper's simultaneous update,
 *   whose decisions may read sites that a neighbouring domain exchanges.  N
 *   attempts per step.
 * Both need N <= 2^31 - 1 and L, H <= 65535.  Energy, clusters,
 * observables, lattice copies, restart and stats work as for
 * kk_create_triangular; kk_get_lattice/kk_set_lattice take N = L*H bytes. */
kk_status kk_create_triangular_ex(kk_sim **out, uint32_t L, uint32_t H, uint32_t scheme, double composition,
                                  double omega_kT, uint64_t seed, void *hip_stream);

/* Whole-sweep tiles of a triangular handle.  Class schedule: with cols > 0
 * every sweep is one launch whose workgroups each own a cols x rows tile and
 * run all 16 classes on an LDS window of the ring around it (33 more sites on
 * every side, recomputed by each tile), writing the tile to the other lattice
 * buffer; cols == 0 selects one launch per class, in place.  Literal MPKK:
 * with cols > 0 every step of 7 iterations is one launch on windows with 21
 * more sites on every side; cols == 0 selects one launch per iteration.
 * Results do not depend on the choice (the window carries every exchange that
 * can reach the tile within the launch).  Needs cols, rows >= 16,
 * cols + 2h <= L, rows + 2h <= H (h = 33, or 21 for MPKK) and a window of at
 * most 143 KiB ((cols + 2h, rounded up to an odd number of 4-byte words) x
 * (rows + 2h) bytes; the workgroup also keeps 16 KiB of queued attempts);
 * KK_EINVAL otherwise and on square handles.  On the
 * class schedule, cols = L and rows = H selects the whole ring in one
 * workgroup's LDS (no halo, up to 1024 sweeps per launch, in place; needs
 * L * H <= 159 KiB).  The default is the tile of least modelled time,
 * ceil(tiles / 256) x ((TW + h')(TR + h') + 4096) with h' = 32 (21 for MPKK),
 * over the square tiles T x T (T = 320, 256, 192, 160, 128, 96, 64, 48, 32,
 * 16) and the tiles that cut the ring into an nx x ny grid (TW = ceil(L/nx),
 * TR = ceil(H/ny), nx, ny <= 64), or 0 when none fits; class-schedule rings
 * of at most 12288 sites default to the whole ring. */
kk_status kk_tri_set_tile(kk_sim *h, uint32_t cols, uint32_t rows);
kk_status kk_tri_get_tile(kk_sim *h, uint32_t *cols, uint32_t *rows);

/* Autotune the tile of a triangular handle (either scheme): time one launch
 * per class (or per MPKK iteration), the handle's current tile, the default
 * tile, every square tile of 320, 256, 192, 160, 128, 96, 64, 48, 32 and 16
 * that fits and the four grid-cut tiles of least modelled time (see
 * kk_tri_set_tile), over trial_sweeps sweeps (0 = 20) after two warm-up
 * sweeps each, and keep the fastest on the handle.  The
 * trials run on the handle's own buffers; its lattice, sweep counter and
 * counters are restored exactly afterwards (results never depend on the tile).
 * Outputs (any may be NULL): the chosen tile (0 x 0 = one launch per class or
 * iteration, L x H = the whole ring in one workgroup, also a candidate) and
 * its time per sweep in microseconds.  Blocking.  KK_EINVAL on
 * a square handle (use kk_autotune). */
kk_status kk_tri_autotune(kk_sim *h, uint32_t trial_sweeps, uint32_t *cols, uint32_t *rows, double *us_per_sweep);

/* Sites per row and rows (H == L except for kk_create_triangular_ex). */
kk_status kk_shape(kk_sim *h, uint32_t *L, uint32_t *H);

/* The 11 thresholds T[0..10] of a triangular handle (KK_EINVAL on a square one). */
kk_status kk_tri_thresholds(kk_sim *h, uint64_t out[11]);

/* 0 for the square torus, 1 for the triangular helical lattice with the
 * conflict-free classes, 2 for the triangular lattice under literal MPKK. */
kk_status kk_geometry(kk_sim *h, uint32_t *geometry);

/* Starting configurations (Results, "MPKK vs. Kawasaki method" and "Cluster
 * Analysis", Figs. 10-11: random against non-random starts). */
enum {
    KK_START_RANDOM = 0,     /* the seeded uniform random subset of kk_create */
    KK_START_SEGREGATED = 1  /* the first n1 sites in index order i = y*L + x hold type 1: full rows
                                0 .. n1/L - 1 and the first n1 % L sites of the next row */
};

/* Put the handle back at a starting configuration of the same size,
 * composition and seed: the lattice is replaced, the sweep counter, attempts
 * and accepted count return to 0.  Works on both geometries and layouts. */
kk_status kk_restart(kk_sim *h, uint32_t start);

/* Run n_sweeps sweeps (N attempts each, the paper's MPKK step), t .. t+n-1,
 * and wait for them.  Advances the sweep counter.  The counter must stay a
 * valid resume point: KK_EINVAL, with nothing run, when t + n_sweeps would
 * reach 2^60 (also for kk_sweep_async, kk_sweep_timed and kk_sweep_series). */
kk_status kk_sweep(kk_sim *h, uint64_t n_sweeps);

/* Enqueue n_sweeps sweeps on the handle's stream and return without waiting.
 * Host-side counters advance immediately; kk_sync waits for the GPU. */
kk_status kk_sweep_async(kk_sim *h, uint64_t n_sweeps);
kk_status kk_sync(kk_sim *h);

/* N_AB (unlike nearest-neighbour bonds over the 2N bonds of the torus) and
 * E/kT = omega * N_AB (the Almeida model, Materials and Methods).  Either
 * output pointer may be NULL. */
kk_status kk_energy(kk_sim *h, uint64_t *n_unlike, double *energy_kT);

/* Cluster-size histogram of `species` (0 or 1): maximal 4-connected periodic
 * sets of sites of that type (the Hoshen-Kopelman analysis of "Cluster
 * Analysis methods", here on the square torus).  Writes up to `cap`
 * (size, count) pairs in ascending size to `out` and the number of distinct
 * sizes to *n_out.  Returns KK_ETRUNC (with *n_out set) when cap is too
 * small; `out` may be NULL when cap == 0. */
kk_status kk_cluster_hist(kk_sim *h, int species, kk_hist_entry *out, size_t cap, size_t *n_out);

/* Observables of the current lattice (Results, "Cluster Analysis": average
 * cluster size over time; Materials and Methods, "Image analysis": the
 * fraction of similar first neighbours).  Every ratio is one correctly
 * rounded division of exact integer sums. */
typedef struct {
    uint64_t sweep;            /* sweep counter t when taken */
    uint64_t n_unlike;         /* N_AB */
    double energy_kT;          /* omega * N_AB */
    double similar_exact;      /* 1 - N_AB / (2N): the fraction of the 2N bonds joining like sites */
    double similar_sampled;    /* random-neighbour estimate: every site draws one of its 4
                                  neighbours (top two bits of its word of Philox block
                                  (y, x / 4, t, tag 5): +x, -x, +y, -y); the fraction of draws
                                  that match its type */
    uint64_t n_clusters;       /* clusters of `species` (as kk_cluster_hist) */
    double size_number_avg;    /* sum s h(s) / sum h(s); 0 without clusters */
    double size_weight_avg;    /* sum s^2 h(s) / sum s h(s); 0 without clusters */
    uint64_t size_max;         /* largest cluster; 0 without clusters */
} kk_observables;

/* Take the observables of the current lattice for `species` (0 or 1). */
kk_status kk_observe(kk_sim *h, int species, kk_observables *out);

/* A time series: count times, run `every` sweeps (every >= 1) and take the
 * observables; out must hold count records. */
kk_status kk_sweep_series(kk_sim *h, uint64_t every, uint64_t count, int species, kk_observables *out);

/* Copy the lattice to host_out (n must be L*L bytes, values 0/1). */
kk_status kk_get_lattice(kk_sim *h, uint8_t *host_out, size_t n);

/* Replace the lattice with host_in (n == L*L bytes, each 0 or 1) and set the
 * sweep counter to sweep_t (< 2^60, KK_EINVAL otherwise): together with
 * kk_get_lattice this is an exact checkpoint/resume, since every random
 * number is addressed by (seed, t, site). */
kk_status kk_set_lattice(kk_sim *h, const uint8_t *host_in, size_t n, uint64_t sweep_t);

/* Sweeps done (= the sweep counter t), attempts made (t' * L * L over the sweeps
 * run by this handle) and exchanges accepted.  NULL outputs are skipped. */
kk_status kk_stats(kk_sim *h, uint64_t *sweeps, uint64_t *attempts, uint64_t *accepted);

/* The 7 acceptance thresholds T[n] = min(2^42, ceil(exp(-omega*(6-2n)) * 2^42)),
 * n = number of unlike neighbours of the pair excluding each other. */
kk_status kk_thresholds(kk_sim *h, uint64_t out[7]);

/* Side length and device layout (KK_LAYOUT_INT8 or KK_LAYOUT_BITPACKED). */
kk_status kk_info(kk_sim *h, uint32_t *L, uint32_t *layout);

/* Override the sweep tile: tile_words x 32 sites wide, tile_rows rows high
 * (even), units_per_thread 1 or 2; tile_words == 0 selects the single cyclic
 * tile holding the whole lattice (needs L % 32 == 0 and at most 1536 row-pair
 * words, (L/2)*(L/32) <= 1536).  Results do not depend on the tile (the decomposition is
 * conflict-free); only speed does. */
kk_status kk_set_tile(kk_sim *h, uint32_t tile_words, uint32_t tile_rows, uint32_t units_per_thread);
kk_status kk_get_tile(kk_sim *h, uint32_t *tile_words, uint32_t *tile_rows, uint32_t *units_per_thread);

/* Autotune the sweep tile: time every candidate (the cyclic tile when it
 * fits; halo tiles 1, 2, 4, 8 or 16 words wide and 32, 48, 64, 96, 128, 192
 * or 256 rows high; one or two units per thread) over trial_sweeps sweeps (0
 * = 20) after a short warm-up, keep the fastest on this handle and use it as
 * the default tile of handles created later in this process with the same L
 * and layout. The trials run on the handle's own buffers; its lattice, sweep
 * counter and counters are restored exactly afterwards (results never depend
 * on the tile). Outputs (any may be NULL): the chosen tile as kk_get_tile
 * reports it and its time per sweep in microseconds. Blocking.
 */
kk_status kk_autotune(kk_sim *h, uint32_t trial_sweeps, uint32_t *tile_words, uint32_t *tile_rows,
                      uint32_t *units_per_thread, double *us_per_sweep);

/* The handle's HIP stream (hipStream_t as void*) for callers that order or time
 * their own work against it. */
kk_status kk_stream(kk_sim *h, void **stream_out);

/* Run n_sweeps sweeps with one HIP event pair on the handle's stream around
 * all of their sweep-kernel launches, which run back to back; *kernel_ms
 * receives the elapsed time between the events (kernel time plus any gaps
 * between launches) and *launches the number of launches.  Blocking.  For
 * profiling; results equal kk_sweep's. */
kk_status kk_sweep_timed(kk_sim *h, uint64_t n_sweeps, double *kernel_ms, uint64_t *launches);

void kk_destroy(kk_sim *h);

/* ---------------------------------------------------------------------------
 * Batches: many independent replicas (uneven L, composition, omega, seed)
 * advanced together.  Replicas with L % 32 == 0 and 64 <= L <= 288 run in
 * persistent launches (one for L <= 160, one for the rest) with the whole
 * lattice held in LDS; the others run as one launch per sweep over all their
 * tiles, replayed from captured HIP graphs.  A replica's result equals what kk_create_ex + kk_sweep gives for the
 * same parameters (no replica or slot index enters any random number).
 * ------------------------------------------------------------------------- */
typedef struct kk_batch kk_batch;

typedef struct {
    uint32_t L;          /* side, as for kk_create */
    uint32_t layout;     /* KK_LAYOUT_* */
    double composition;  /* fraction of type 1, in [0, 1] */
    double omega_kT;     /* interaction omega / kT, finite */
    uint64_t seed;       /* Philox key */
    uint64_t sweeps;     /* sweeps this replica makes on every kk_batch_run (at most 2^31 - 1) */
    uint32_t start;      /* KK_START_RANDOM (0, kk_create's start) or KK_START_SEGREGATED */
} kk_replica;

/* Create n replicas (each placed as kk_create would, then put at its start as
 * kk_restart would) on one device; hip_stream (NULL = own) carries the uploads
 * and the tiled launches.  KK_EINVAL for an unknown start. */
kk_status kk_batch_create(kk_batch **out, const kk_replica *reps, size_t n, void *hip_stream);

/* Advance every replica by its `sweeps` and wait. */
kk_status kk_batch_run(kk_batch *b);

/* Borrow replica i's handle for queries (kk_get_lattice, kk_energy,
 * kk_cluster_hist, kk_stats, ...).  kk_set_lattice on it between runs is
 * allowed: every run starts from the handle's lattice and sweep counter.
 * The batch owns it: do not destroy it. */
kk_status kk_batch_sim(kk_batch *b, size_t i, kk_sim **sim_out);

/* The cluster-size histogram of `species` (0 or 1) of every replica, the one
 * kk_cluster_hist gives (Materials and Methods, "Cluster Analysis methods":
 * the statistics taken regularly during a run), computed for all replicas
 * with one wait on the device instead of one per replica.  The results are
 * held by the replicas' handles: kk_cluster_hist on a borrowed handle then
 * returns them without device work until the replica's lattice changes.
 * KK_EINVAL for another species, KK_ESTATE for a poisoned batch or replica,
 * KK_EDEVICE (batch poisoned) on a device error.  Blocking. */
kk_status kk_batch_cluster_hists(kk_batch *b, int species);

/* Autotune the tiles of the tiled replicas: time whole batch runs of
 * trial_sweeps sweeps (0 = 10) for tiles (words x at most rows) of
 * 8 x 128, 16 x 84, 8 x 64, 16 x 42, 8 x 32 and 8 x 16 at two units per
 * thread, and 16 x 28, 16 x 20, 8 x 72, 8 x 50 and 8 x 32 at one unit per
 * thread (smaller tiles give more workgroups when the batch holds little
 * work, larger ones less halo work), keep the fastest and re-plan.
 * Every replica's lattice, sweep counter and counters are restored exactly
 * after the trials.  Outputs (any may be NULL): the chosen maximum tile width
 * (words) and height (rows) and the best trial's milliseconds per sweep.
 * Blocking. */
kk_status kk_batch_autotune(kk_batch *b, uint32_t trial_sweeps, uint32_t *tile_words, uint32_t *tile_rows,
                            double *ms_per_sweep);

/* Set the tile caps of the tiled replicas by hand (words 8 or 16; rows even,
 * at most 128; 1 or 2 units per thread; a tile of (rows + 28) / 2 row pairs
 * of words + 2 words must fit 512 threads times the units per thread) and
 * re-plan, e.g. to repeat a tile that kk_batch_autotune chose.  Results never
 * depend on the tile.  KK_EINVAL for a cap outside these limits. */
kk_status kk_batch_set_tile(kk_batch *b, uint32_t tile_words, uint32_t tile_rows, uint32_t units_per_thread);

/* How the batch runs: resident replicas, tiled replicas, tile jobs per sweep. */
kk_status kk_batch_info(kk_batch *b, size_t *n_resident, size_t *n_tiled, size_t *n_tile_jobs);

void kk_batch_destroy(kk_batch *b);

/* ---- Batches of triangular lattices ----------------------------------
 * Many replicas of the triangular helical lattice (the paper's model),
 * advanced together.  When at least 64 class-schedule replicas have rings of
 * at most 159 KiB, those run "resident": one launch per run, one workgroup per
 * replica holding its whole ring in LDS for all of its sweeps.  Other
 * class-schedule replicas whose lattice takes a whole-sweep tile are
 * "batched": each sweep of a run is one launch whose workgroups are the tiles
 * of all batched replicas that still have sweeps to make.  Literal-MPKK
 * replicas and the rest run through their own launches on the batch stream.
 * A replica's result equals what kk_create_triangular_ex + kk_restart(start)
 * + kk_sweep(sweeps) per run gives alone (no replica index enters a random
 * counter). */
typedef struct kk_tri_batch kk_tri_batch;

typedef struct {
    uint32_t L;          /* sites per row, as for kk_create_triangular_ex */
    uint32_t H;          /* rows */
    uint32_t scheme;     /* KK_TRI_CLASSES or KK_TRI_MPKK */
    uint32_t start;      /* KK_START_RANDOM or KK_START_SEGREGATED */
    double composition;  /* fraction of type 1, in [0, 1] */
    double omega_kT;     /* omega / kT, finite */
    uint64_t seed;       /* Philox key */
    uint64_t sweeps;     /* sweeps (MPKK: steps) of this replica on every kk_tri_batch_run, at most 2^31 - 1 */
} kk_tri_replica;

/* Create n replicas (validated and placed as kk_create_triangular_ex and
 * kk_restart would) on one device; hip_stream (NULL = own) carries all of
 * their work.  *out receives the batch (NULL on failure). */
kk_status kk_tri_batch_create(kk_tri_batch **out, const kk_tri_replica *reps, size_t n, void *hip_stream);
/* Advance every replica by its sweeps; blocking. */
kk_status kk_tri_batch_run(kk_tri_batch *b);
/* Borrow replica i's handle (owned by the batch: query it, copy its lattice,
 * never destroy it). */
kk_status kk_tri_batch_sim(kk_tri_batch *b, size_t i, kk_sim **sim_out);
/* Resident replicas (whole ring in one workgroup), replicas in the batched
 * tile launch, replicas run on their own, and tile jobs of the batched
 * launch.  NULL outputs are skipped. */
kk_status kk_tri_batch_info(kk_tri_batch *b, size_t *n_resident, size_t *n_batched, size_t *n_plain,
                            size_t *n_jobs);
void kk_tri_batch_destroy(kk_tri_batch *b);

/* ---------------------------------------------------------------------------
 * Job server: independent simulation jobs (a kk_replica each, `sweeps` being
 * the job's total) arrive at any time and are served on one device.
 *
 *  - Admission: jobs wait in arrival (FIFO) order until their device memory
 *    fits hbm_budget_bytes next to the jobs already admitted and a slot of
 *    max_active is free.  A job's charge is an upper bound of what it holds:
 *    two lattice buffers plus 8 bytes per site (placement keys, later the
 *    cluster labels) plus small tables.  A job that alone exceeds the budget
 *    is refused at submission (KK_ENOMEM).
 *  - Continuous batching: each kk_server_step advances every admitted job by
 *    min(chunk_sweeps, sweeps left) sweeps in one batch run (the batch engine
 *    above), retires the jobs that are done and admits waiting ones; jobs join
 *    and leave only between steps.
 *  - Results: for a finished job, N_AB and E/kT = omega * N_AB of the final
 *    lattice, the accepted-move count and the cluster-size histogram of
 *    species 1 (as kk_cluster_hist), plus the final lattice if keep_lattice
 *    is set.  Each equals what kk_create_ex + kk_sweep(sweeps) gives for the
 *    job alone, whatever else runs beside it.
 *  - Times are seconds on the server's monotonic clock (kk_server_now; zero at
 *    creation).  Latency = t_done - t_arrival.
 * The server is driven by one host thread; calls on one server must not
 * overlap.  Paper: the many short and long simulations its kinetic study
 * needs (section "Results"), served together; this is the throughput side of
 * the method, not a step of it.
 * ------------------------------------------------------------------------- */
typedef struct kk_server kk_server;

typedef struct {
    uint64_t hbm_budget_bytes; /* device bytes admitted jobs may hold together; 0 = 3/4 of free memory */
    uint32_t max_active;       /* jobs advanced together; 0 = 256 */
    uint32_t keep_lattice;     /* nonzero: keep each finished lattice on the host */
    uint64_t chunk_sweeps;     /* sweeps per step; 0 = 1000; below 2^31 */
    void *hip_stream;          /* hipStream_t for uploads and joins; NULL = own */
} kk_server_config;

typedef struct {
    uint64_t id;
    int32_t status;            /* KK_OK, or the error that ended the job */
    uint32_t L;
    uint64_t sweeps, attempts, accepted;
    uint64_t n_unlike;         /* N_AB of the final lattice */
    double energy_kT;          /* omega * N_AB */
    double t_arrival, t_admit, t_done;
    uint64_t hist_entries;     /* entries of the species-1 cluster histogram */
} kk_job_result;

typedef struct {
    uint64_t submitted, admitted, completed, steps;
    uint64_t queued, active;
    uint64_t bytes_in_use, peak_bytes, budget;
    uint64_t attempts;         /* attempts made by all steps so far */
    double gpu_busy_s;         /* wall time spent inside batch runs */
} kk_server_stats;

/* cfg may be NULL (all defaults). */
kk_status kk_server_create(kk_server **out, const kk_server_config *cfg);

/* Current time on the server clock. */
kk_status kk_server_now(kk_server *s, double *t);

/* The device bytes a job is charged at admission (an upper bound of what it
 * holds at any time): two lattice buffers, the energy counters and one
 * accepted-move sum per sweep tile, plus the larger of the placement scratch
 * (8 bytes per site and the radix tables) and the retirement scratch (the
 * cluster-labelling arrays, 8 bytes per site and the size tables, and with
 * keep_lattice on a bit-packed job the N-byte unpack buffer of the lattice
 * copy), plus 64 KiB for the job's share of the batch tables.  Host-only: no
 * device call.  KK_EINVAL for a NULL argument, a bad L or layout. */
kk_status kk_server_job_bytes(const kk_replica *job, uint32_t keep_lattice, uint64_t *bytes);

/* Queue a job (validated as kk_create_ex would, plus the budget check).
 * arrival_s < 0 stamps the arrival now; otherwise it is taken as given (a
 * trace replayer passes the scheduled arrival).  *job_id receives the id. */
kk_status kk_server_submit(kk_server *s, const kk_replica *job, double arrival_s, uint64_t *job_id);

/* Admit, advance every admitted job by one chunk (blocking), retire finished
 * jobs, admit again.  Returns the admitted and waiting counts. */
kk_status kk_server_step(kk_server *s, size_t *n_active, size_t *n_queued);

/* Move up to cap finished, not yet polled results into out (completion
 * order); *n_out receives the number written (the rest stay for later). */
kk_status kk_server_poll(kk_server *s, kk_job_result *out, size_t cap, size_t *n_out);

/* A finished job's species-1 histogram (ascending size); KK_ETRUNC with
 * *n_out = the entry count when cap is too small. */
kk_status kk_server_job_hist(kk_server *s, uint64_t job_id, kk_hist_entry *out, size_t cap, size_t *n_out);

/* A finished job's final lattice as L*L bytes of 0/1 (needs keep_lattice). */
kk_status kk_server_job_lattice(kk_server *s, uint64_t job_id, uint8_t *out, size_t n);

/* Drop a finished, polled job's host-side results. */
kk_status kk_server_release(kk_server *s, uint64_t job_id);

kk_status kk_server_get_stats(kk_server *s, kk_server_stats *out);

/* Frees every job, queued, running or finished. */
void kk_server_destroy(kk_server *s);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sweeps
 * of kk_sweep on a square-torus lattice that the caller holds in device
 * memory, with no allocation of any kind.
 *   lattice   device pointer, in and out: KK_LAYOUT_INT8 (L*L bytes, 0/1,
 *             row-major) or KK_LAYOUT_BITPACKED (L rows of L/32 uint32, bit b
 *             of word g = site 32g + b); owned by the caller.
 *   omega_kT, seed  as for kk_create; t0 = the first sweep's counter, so that
 *             a handle at counter t0 holding the same lattice reaches the
 *             same state with kk_sweep(n_sweeps), bit for bit.
 *   accepted  device pointer (may be NULL): the accepted exchanges of these
 *             sweeps are ADDED to *accepted.
 *   hip_stream  the stream to enqueue on (NULL = the null stream).
 * The call enqueues its work and returns without waiting.  The second lattice
 * buffer and the per-tile counts live in a fixed device array of
 * KK_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends: lattices up
 * to 8 MiB (bit-packed L <= 8192, int8 L <= 2896) and at most 4096 sweep
 * tiles; larger inputs give KK_EINVAL.  Every call on one GPU shares that
 * array, so calls whose work overlaps on one GPU (other streams, other
 * threads) race: serialise them.  KK_EINVAL also for a NULL lattice, a bad L
 * or layout (L % 4 == 0; bit-packed L % 32 == 0), non-finite omega or
 * t0 + n_sweeps >= 2^60; KK_EDEVICE for a failed launch. */
#define KK_NOALLOC_SCRATCH_BYTES ((size_t)8 * 1048576 + (size_t)4096 * 8)
kk_status kk_sweep_noalloc(void *lattice, uint32_t L, uint32_t layout, double omega_kT, uint64_t seed, uint64_t t0,
                           uint64_t n_sweeps, unsigned long long *accepted, void *hip_stream);

/* Measurement aid for pricing the kernels' VALU roofline: the SIMD cycles one
 * wave64 instruction of each kind below occupies on the current device, from
 * timed probe kernels (eight independent chains per lane, 32 waves per CU),
 * the device's CU count (4 SIMDs each) and its reported clock.  out[i] for
 * i = KK_VALU_XOR, _BITOP3, _ALIGNBIT, _ADD, _MAD_U64_U32, _MUL_LO, _FMA_F32,
 * _LSHL, _BCNT.
 * Allocates a small buffer and blocks; KK_EDEVICE on a failed launch. */
enum {
    KK_VALU_XOR = 0, KK_VALU_BITOP3 = 1, KK_VALU_ALIGNBIT = 2, KK_VALU_ADD = 3,
    KK_VALU_MAD_U64_U32 = 4, KK_VALU_MUL_LO = 5, KK_VALU_FMA_F32 = 6, KK_VALU_LSHL = 7, KK_VALU_BCNT = 8,
    KK_VALU_PROBES = 9
};
kk_status kk_valu_issue_cycles(double out[KK_VALU_PROBES]);

/* Message of the last error on the calling thread ("" if none). */
const char *kk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KK_H */
