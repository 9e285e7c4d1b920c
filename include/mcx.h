/*
 * mcx.h - C ABI of libmcx: event-based Monte Carlo neutron transport for
 * k-eigenvalue power iteration on one AMD Instinct MI355X (gfx950).
 *
 * The method is the one the paper studies (Morgan, Cuneo, Variansyah,
 * Niemeyer, M&C 2025, arXiv 2501.05440): Sec. 1 names the physics
 * (multigroup energy, constructive solid geometry with surface tracking,
 * k-eigenvalue power iteration, replicable CPU/GPU random numbers); Sec. 2
 * names the event-based GPU structure (particles taken from a
 * to-be-processed bank, written to a processed bank, events launched as
 * separate kernels); Sec. 5 fixes FP64 arithmetic.  Each generation runs
 * birth, then repeated {advance: cross-section lookup, distance to
 * collision, distance to boundary, move, track-length tallies, surface
 * crossing} and {collide: fission-bank append, absorption or scatter}
 * kernels over compacted particle banks, then builds the canonical fission
 * bank, the k estimators, the Shannon entropy and the next source.
 *
 * Conventions
 *  - Every call returns MCX_OK (0) or a negative MCX_E* code and never
 *    aborts; mcx_last_error() gives a message for the context.
 *  - Host arrays passed to mcx_load_* / mcx_seed_source are copied before
 *    the call returns; the caller may free them afterwards.
 *  - The device workspace and the stream belong to the caller.  The library
 *    never allocates or frees device memory; it carves the bound workspace.
 *  - Output arrays of mcx_get_* are caller-allocated host memory.
 *  - Call order: create -> load_geometry, load_mg_xs, seed_source (any
 *    order) -> workspace_size -> bind_workspace -> run_generations ->
 *    get_* -> destroy.  Loading or seeding again requires binding again.
 *  - Not thread-safe per context; distinct contexts are independent.
 */
#ifndef MCX_H
#define MCX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mcx_ctx mcx_ctx;

enum mcx_status {
  MCX_OK = 0,
  MCX_EINVAL = -1,     /* invalid argument or problem data */
  MCX_ESTATE = -2,     /* call out of order */
  MCX_ENOMEM = -3,     /* workspace too small, or host allocation failed */
  MCX_EDEVICE = -4,    /* HIP runtime error */
  MCX_ELOST = -5,      /* source sampling found no fissile point */
  MCX_EGUARD = -6,     /* histories stopped by the per-history event guard */
  MCX_EEXTINCT = -7,   /* empty fission bank in a k-eigenvalue generation */
  MCX_EOVERFLOW = -8   /* fission bank or per-history site count overflow, or 2^32
                          flights or more in one generation or batch (the limit
                          of the exact flux accumulators) */
};

enum { MCX_FP64 = 0, MCX_FP32_MIXED = 1 };
enum {
  MCX_ENGINE_EVENT = 0,
  MCX_ENGINE_PERSISTENT = 1,
  MCX_ENGINE_MONOLITHIC = 2,
  MCX_ENGINE_ASYNC = 3
};
enum { MCX_VACUUM = 0, MCX_REFLECT = 1 };
enum {
  MCX_FATE_ABSORBED = 1,
  MCX_FATE_LEAKED = 2,
  MCX_FATE_KILLED = 3,
  MCX_FATE_CUTOFF = 4,
  MCX_FATE_CENSUS = 5
};

/* Per-generation counters, in this order (mcx_get_generation_stats). */
enum {
  MCX_CNT_SEG = 0,    /* flight segments = collisions + crossings */
  MCX_CNT_COL = 1,    /* collisions */
  MCX_CNT_CROSS = 2,  /* surface crossings (reflections and leaks included) */
  MCX_CNT_REFL = 3,   /* crossings with a reflection */
  MCX_CNT_LEAK = 4,   /* histories ended by leakage */
  MCX_CNT_ABS = 5,    /* histories ended by absorption */
  MCX_CNT_KILLED = 6, /* histories ended by the event guard */
  MCX_CNT_SITES = 7,  /* fission sites banked */
  MCX_CNT_SCAT = 8,   /* scatters */
  MCX_CNT_CUTOFF = 9, /* histories ended below the energy cutoff (continuous energy) */
  MCX_CNT_CENSUS = 10, /* histories that reached the end of the time grid (time-dependent) */
  MCX_N_CNT = 11
};

typedef struct {
  int32_t precision;        /* MCX_FP64 (the paper's precision, Sec. 5) */
  int32_t device;           /* HIP device ordinal the workspace lives on */
  void* stream;             /* hipStream_t for every launch and copy; NULL = null stream */
  int32_t block_size;       /* threads per block of the event kernels, multiple of 64; 0 = 512
                               (multigroup) or 256 (continuous energy) */
  int32_t tail_threshold;   /* live-particle count at or below which one history-based
                               kernel finishes the generation; 0 = default
                               (n_per_gen / 8 within [4096, 131072]); negative = event
                               kernels until every history ends */
  int32_t lookahead;        /* event iterations enqueued ahead of the last live count
                               read back; 0 = default (4) */
  int64_t max_events;       /* per-history segment guard; 0 = 100000 */
  int32_t record_histories; /* 1: keep one mcx_record per history per generation */
  int32_t time_kernels;     /* 1: time every event kernel with HIP events (mcx_get_timing);
                               2: time only the advance kernels (fewer events between
                               launches, each of which delays the next launch a little) */
  /* Engine.  MCX_ENGINE_EVENT launches one kernel per event class and
     iteration over banks compacted in device memory (the structure of the
     paper's Sec. 2).  MCX_ENGINE_PERSISTENT runs each generation (or batch)
     as one kernel whose workgroups keep particles in LDS slots, process them
     event by event over block-local queues, and refill free slots from a
     global history counter; batches (mcx_load_batch) always use it.
     MCX_ENGINE_MONOLITHIC is the paper's monolithic event (Sec. 2): each
     launch runs one whole segment of every live particle (flight, then its
     collision or crossing, in one kernel) from a to-be-processed bank into a
     processed bank, with no sorting and no history-based tail, until every
     history has ended; block_size, lookahead, record_histories and
     time_kernels apply (its launches count as advance launches), flights
     and tail_threshold do not.  MCX_ENGINE_ASYNC is an asynchronous
     schedule (Sec. 2 names the runtime's asynchronous scheduler beside the
     event-based one): one launch per generation (or batch) whose workgroups
     keep pulling blocks of particles from two global queues, one per event
     type (advance, collide), or give birth to the next histories, and push
     every survivor to the queue of its next event, with no grid-wide
     barrier; particle state lives in a global pool.  p_grid sets its
     workgroups and flights its flights per advance item; multigroup only,
     FP64 or FP32-mixed, batches included.  Every engine gives identical
     per-history results.  record_histories requires the event or
     monolithic engine. */
  int32_t engine;
  int32_t p_block;          /* persistent: threads per block, 128 or 256; 0 = 256 */
  int32_t p_slots;          /* persistent: particle slots per block, 256 or 512; 0 = 512 */
  int32_t p_grid;           /* persistent and asynchronous engines: workgroups;
                               0 = 2 per compute unit (persistent), 1 per 2 compute
                               units (asynchronous) */
  double p_tau;             /* persistent: refill when fewer than p_tau * p_slots particles
                               of a block are live, 0 < p_tau <= 1; 0 = 0.75 */
  int32_t p_sort;           /* persistent: 1 = order each collide list by material class
                               (fissile first) so fission sampling runs in the same waves */
  int32_t flights;          /* event and asynchronous engines: flights one advance step
                               makes per particle
                               before it returns to the live bank (it stops earlier at a
                               collision, a leak or the guard).  1 = one event per launch,
                               the paper's decomposition; larger values keep a particle in
                               the kernel across surface crossings.  Results are identical
                               for every value.  0 = default (8); at most 65536 */
  int32_t event_log;        /* > 0 (with record_histories = 1): keep the first event_log
                               flights of every history in every generation as mcx_event
                               entries (mcx_get_event_log); at most 65536 */
  int32_t time_stride;      /* with time_kernels: time the launches of generations
                               g % time_stride == 0 only (the timing events of the
                               others are left out); 0 or 1 = every generation */
  int32_t rounds;           /* event engine (multigroup): particles per thread of an
                               advance block.  1 = one particle per thread; r > 1: a
                               block owns r x block_size particles and a lane whose
                               particle stops takes the next one, so lanes do not idle
                               behind the wave's longest chain of crossings
                               (r x block_size <= 4096).  Results are identical for
                               every value.  0 = default */
  int32_t lds_tally_min;    /* event engine (multigroup, tables small enough for LDS): an
                               advance launch whose live-count bound is at least this
                               stages its flux tally in LDS (each 768-thread block keeps
                               16 B per tally bin and adds every bin to device memory once,
                               instead of one device atomic per flight) when the device's
                               LDS per block holds it.  Results are identical either way.
                               0 = default (2^19); negative = never */
  int32_t lt_flights;       /* flights per particle of those LDS-staged advance launches
                               (the large ones; `flights` applies to the others).  Results
                               are identical for every value.  0 = default
                               (min(flights, 5)); at most 65536 */
} mcx_options;

/* Lattice of pin universes (paper Sec. 1: CSG geometry).  Cell (i, j),
   0 <= i < nx, 0 <= j < ny, spans [x0 + i pitch, x0 + (i+1) pitch] x
   [y0 + j pitch, y0 + (j+1) pitch]; universe u has n_rings[u] concentric
   z-cylinders about the cell centre with strictly increasing radii below
   pitch / 2; region r < n_rings[u] is inside ring r (and outside ring r-1),
   region n_rings[u] is outside every ring; its material is
   mats[u * (max_rings + 1) + r].  bc = {xmin, xmax, ymin, ymax} sides, each
   MCX_VACUUM or MCX_REFLECT.  Limits: nx, ny <= 4095, max_rings <= 254. */
typedef struct {
  int32_t nx, ny;
  double pitch, x0, y0;
  int32_t bc[4];
  int32_t n_univ, max_rings;
  const int32_t* n_rings;   /* [n_univ] */
  const double* radii;      /* [n_univ][max_rings] */
  const int32_t* mats;      /* [n_univ][max_rings + 1] */
  const int32_t* pin_map;   /* [ny][nx] universe of each cell */
} mcx_geometry;

/* Source and run description.  The generation-0 source (and every batch of
   a fixed-source run) is uniform over the fissile volume with a group drawn
   from the fission spectrum.  fixed_source = 1 treats fission as capture
   (production is tallied, no sites are banked) and samples a fresh source
   every batch.  problem_id enters every random-number counter, so a problem
   run alone or inside a batch sees the same streams.  The entropy mesh
   (ent_nx x ent_ny) covers the lattice's bounding box. */
typedef struct {
  uint64_t seed;
  int64_t n_per_gen;        /* 1 <= n_per_gen <= 2^30 */
  int32_t fixed_source;
  uint64_t problem_id;
  int32_t ent_nx, ent_ny;
} mcx_source;

/* Per-history record (record_histories = 1). */
typedef struct {
  int32_t n_seg, n_col, n_cross, n_refl;
  int32_t fate, n_sites, g_final;
  uint32_t ctr_final;       /* transport-stream draws consumed */
  double tl_sum;            /* total track length */
  double kcol_sum;          /* sum of nu_sig_f / sig_t over collisions */
  double x_final, y_final;
  double e_final;           /* final energy (continuous energy), else 0 */
  double t_final;           /* final time (time-dependent mode), else 0 */
} mcx_record;

/* One logged flight (event_log > 0): position after it, its length, the
   energy it flew at (continuous energy, else 0), the lattice cell
   (j * nx + i), ring region and group or energy bin it flew in, and how it
   ended: 1 collision, 2 surface crossing, 3 leak, 4 census.  Unused entries
   are 0. */
typedef struct {
  double x, y, d, e;
  int32_t cell, region, group, type;
} mcx_event;

/* Timing of the last mcx_run_generations or mcx_run_batch.  The *_ms kernel sums are filled
   when time_kernels = 1 (events recorded on the stream around each launch; with
   time_kernels = 2 only advance_ms / n_advance; with time_stride > 1 over the timed
   generations only, while the *_items, advance_segments and n_iterations count all);
   *_items count the particles each kernel class processed. */
typedef struct {
  double run_ms;            /* stream time of the whole run, generation ends included */
  int64_t n_iterations;     /* advance + collide iterations launched */
  int64_t n_tail_launches;
  double advance_ms, collide_ms, tail_ms;
  int64_t n_advance, n_collide;
  int64_t advance_items;    /* particles processed by advance kernels (= their segments + kills) */
  int64_t collide_items;    /* collisions processed by collide kernels */
  double persistent_ms;     /* persistent-engine kernels (time_kernels = 1) */
  int64_t n_persistent;
  int64_t advance_segments; /* flights made inside advance kernels */
} mcx_timing;

/* One problem of a batch: its lattice, multigroup data (as for
   mcx_load_geometry and mcx_load_mg_xs, material indices local to the
   problem), random-number seed and problem id, and history count.  A batch
   problem is a single fixed-source generation (fission treated as capture,
   production tallied), with the source of mcx_source; problem_id keys its
   random numbers exactly as in a single-problem run, so a problem gives the
   same histories inside a batch and alone. */
typedef struct {
  mcx_geometry geo;
  int32_t n_mat, n_grp;
  const double* sig_t;
  const double* sig_s;
  const double* nu_sig_f;
  const double* chi;
  uint64_t seed;
  int64_t n_hist;           /* >= 1 */
  uint64_t problem_id;
} mcx_problem;

/* Launch configuration picked by mcx_autotune.  Persistent engine: block,
   slots, grid, tau, sort.  Event engine: block (block_size), flights,
   lt_flights and tail (tail_threshold); the other fields are 0. */
typedef struct {
  int32_t block, slots, grid;
  double tau;
  double ms;                /* measured stream time of one batch (or generation) */
  int32_t sort;             /* collide lists ordered by material class */
  int32_t flights, lt_flights, tail;
} mcx_tune;

/* Create a context on opt->device (NULL opt = defaults).  Project addition,
   no passage: the paper's runs are driven from Python (Sec. 3). */
int mcx_create(mcx_ctx** out, const mcx_options* opt);

/* Copy and validate the geometry (paper Sec. 1: constructive solid geometry
   with surface tracking; MCX_EINVAL on bad sizes, radii, pin map). */
int mcx_load_geometry(mcx_ctx* ctx, const mcx_geometry* geo);

/* Copy and validate multigroup data (paper Sec. 1: multigroup physics):
   sig_t[m][g] > 0; sig_s[m][g][g'] >= 0 is the transfer g -> g' with
   sum_g' sig_s <= sig_t; nu_sig_f[m][g] >= 0; chi[m][g] >= 0 summing to
   about 1 for every fissile material.  1 <= n_grp <= 65535. */
int mcx_load_mg_xs(mcx_ctx* ctx, int32_t n_mat, int32_t n_grp, const double* sig_t,
                   const double* sig_s, const double* nu_sig_f, const double* chi);

/* Continuous-energy data (paper Sec. 1: continuous-energy physics; Sec. 4:
   continuous-energy pin cell).  Pointwise microscopic cross sections on one
   shared, strictly increasing energy grid, interpolated linearly in energy
   (the interval is the largest i with e_grid[i] <= E, within [0, n_pts-2];
   the fraction is clipped to [0, 1]); a material's macroscopic value is the
   density-weighted sum over its nuclides in the listed order.  A collision
   banks floor(nu Sigma_f / (Sigma_t k) + xi) sites with Watt energies,
   picks the nuclide by its share of Sigma_t, then scatters elastically off
   it (target at rest, isotropic in the centre-of-mass frame, direction
   turned about itself) or absorbs; a scatter below e_cut ends the history
   (MCX_FATE_CUTOFF).  The flux is tallied per (cell, region, energy bin)
   with n_ebins bins between e_edges; the production tally is not kept
   (reads zero) and the track-length k estimator is summed directly.
   Event engine, FP64 and FP32-mixed. */
typedef struct {
  int32_t n_nuc, n_pts;
  const double* e_grid;     /* [n_pts] eV */
  const double* sig_t;      /* [n_nuc][n_pts] barns; sig_t >= sig_s */
  const double* sig_s;      /* [n_nuc][n_pts] elastic scattering */
  const double* sig_f;      /* [n_nuc][n_pts] fission */
  const double* awr;        /* [n_nuc] target mass / neutron mass, > 0 */
  double nu;                /* neutrons per fission */
  int32_t n_mat, max_nuc;
  const int32_t* mat_n;     /* [n_mat] nuclides per material, 1..max_nuc */
  const int32_t* mat_nuc;   /* [n_mat][max_nuc] */
  const double* mat_dens;   /* [n_mat][max_nuc] atoms per barn-cm, >= 0 */
  double watt_a, watt_b;    /* Watt spectrum, eV and 1/eV: E = W + a^2 b/4 +
                               (2 xi - 1) sqrt(a^2 b W), W Maxwellian of temperature a */
  double e_max;             /* Watt energies above e_max are drawn again */
  double e_cut;             /* energy cutoff, eV */
  int32_t n_ebins;
  const double* e_edges;    /* [n_ebins + 1] strictly increasing, eV */
  double src_energy;        /* > 0: every source particle starts at this energy (eV;
                               the paper's time-dependent pin cell uses 14 MeV,
                               Sec. 4); 0: Watt spectrum */
} mcx_ce_data;

/* Copy and validate continuous-energy data (paper Sec. 1: continuous-energy
   physics; Sec. 4: continuous-energy pin cell); replaces multigroup data. */
int mcx_load_ce_xs(mcx_ctx* ctx, const mcx_ce_data* ce);

/* Time-dependent fixed source (paper Sec. 1: MC/DC's time-dependent mode;
   Sec. 4 runs the continuous-energy pin cell in it): every history starts
   at t = 0 from the fixed source (mcx_source with fixed_source = 1, fission
   treated as capture); a flight of length d lasts d / v, v = speed[g] for
   multigroup data and, for continuous energy, the speed of a neutron of the
   flight's energy, c sqrt(2 E / m c^2) (c = 2.99792458e10 cm/s,
   m c^2 = 939.56542052e6 eV); the flux tally gains n_tbins time bins (bin
   index * n_tbins + time bin), each flight adding the length it flies
   inside each bin; a history still flying at t_edges[n_tbins] stops there
   (MCX_FATE_CENSUS).  For continuous energy the production tally holds the
   neutron density instead: the time spent per bin per source particle, in
   seconds.  t_edges[0] = 0, strictly increasing; multigroup: speed in cm/s,
   one per group (n_grp must match the loaded data at bind time);
   continuous energy: speed = NULL and n_grp = 0.  Event or monolithic
   engine.  n_tbins = 0 switches the mode off. */
int mcx_load_time_grid(mcx_ctx* ctx, int32_t n_tbins, const double* t_edges,
                       const double* speed, int32_t n_grp);

/* Set the random-number seed, histories per generation and the source of
   the run (paper Sec. 1: k-eigenvalue and fixed-source modes, random numbers
   replicable between CPU and GPU). */
int mcx_seed_source(mcx_ctx* ctx, const mcx_source* src);

/* Bytes of device workspace needed to run up to n_gen_max generations.
   Project addition, no passage (caller-owned device memory). */
int mcx_workspace_size(mcx_ctx* ctx, int32_t n_gen_max, size_t* bytes);

/* Bind a caller-owned device buffer (256-byte aligned, on opt->device) of at
   least mcx_workspace_size bytes and upload the tables; MCX_ENOMEM if small.
   Project addition, no passage. */
int mcx_bind_workspace(mcx_ctx* ctx, void* device_ptr, size_t bytes, int32_t n_gen_max);

/* Power iteration (paper Sec. 4: inactive then active cycles): n_gen
   generations, statistics over the last n_gen - n_inactive.  Blocks until
   the stream has finished.  Returns MCX_EEXTINCT, MCX_EOVERFLOW, MCX_ELOST,
   MCX_EGUARD (results are still readable) or MCX_EDEVICE on failure. */
int mcx_run_generations(mcx_ctx* ctx, int32_t n_gen, int32_t n_inactive);

/* Bytes of the library's static per-device scratch array used by
   mcx_run_generations_noalloc. */
#define MCX_SCRATCH_BYTES (64u * 1024u * 1024u)

/* mcx_run_generations for callers that cannot allocate device memory (code
   under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc): binds the library's static scratch array of this GPU
   (MCX_SCRATCH_BYTES, held until the process ends) as the context's
   workspace, sized for n_gen generations, uploads the tables into it and
   runs the generations; it calls no hipMalloc, hipFree, hipHostMalloc or
   other device or pinned-memory allocator.  The caller still creates,
   loads and seeds the context; results are read with the usual getters.
   MCX_ENOMEM (with the byte counts in mcx_last_error) if the run needs more
   than MCX_SCRATCH_BYTES; MCX_EINVAL with time_kernels on (timing creates
   events) or bad generation counts; MCX_ESTATE for a batch or before
   loading and seeding; otherwise as mcx_run_generations.  Every context on
   one GPU shares that GPU's array, which keeps the last call's contents: a
   later call (from any context) overwrites the workspace of the earlier
   one, and calls that overlap on one GPU race.  The context stays bound to
   the array afterwards (mcx_continue_generations and the getters read it),
   until it is bound again. */
int mcx_run_generations_noalloc(mcx_ctx* ctx, int32_t n_gen, int32_t n_inactive);

/* Continue the last completed run (or a restored checkpoint) by n_more
   generations: the next generation starts from the source and k_used the
   previous one left, with the same random streams, so a run continued in
   pieces equals one uninterrupted run of the total length.  Statistics
   cover every generation so far with the first run's n_inactive.  The total
   must stay within n_gen_max.  Project addition, no passage. */
int mcx_continue_generations(mcx_ctx* ctx, int32_t n_more);

/* Serialize the state a continued run needs after a completed run: the next
   source, k_used and every generation's results so far (not the per-history
   records), tied to the problem, precision and event guard by a
   fingerprint.  buf = NULL: *len receives the size in bytes.  MCX_ENOMEM if
   *len is too small (then *len receives the size).  Project addition, no
   passage. */
int mcx_checkpoint(mcx_ctx* ctx, void* buf, size_t* len);

/* Load a checkpoint into a context bound to the same problem (MCX_EINVAL
   otherwise); the results read back as after the checkpointed run, and
   mcx_continue_generations proceeds from it.  Project addition, no passage. */
int mcx_restore(mcx_ctx* ctx, const void* buf, size_t len);

/* k-eigenvalue estimates (paper Sec. 1: k-eigenvalue power iteration; Sec. 4:
   inactive then active cycles): active-generation mean and standard
   deviation of the mean of the collision, track-length and absorption k
   estimators (mean3, sigma3), and
   optionally the per-generation values per_gen[n_gen][3] (may be NULL). */
int mcx_get_keff(mcx_ctx* ctx, double* mean3, double* sigma3, double* per_gen);

/* Per-generation Shannon entropy of the fission bank entropy[n_gen] and
   counters counts[n_gen][MCX_N_CNT]; either may be NULL.  Project addition,
   no passage (convergence and balance diagnostics of the power iteration,
   Sec. 4). */
int mcx_get_generation_stats(mcx_ctx* ctx, double* entropy, int64_t* counts);

/* Tallies (paper Sec. 2: the transport loop's tally operations):
   active-generation mean and standard deviation of the mean of the
   track-length flux and nu-fission production per source particle, bin
   ((cell j * nx + i) * (max_rings + 1) + region) * n_grp + group; n_bins must
   equal nx * ny * (max_rings + 1) * n_grp.  Any pointer may be NULL. */
int mcx_get_tallies(mcx_ctx* ctx, double* flux_mean, double* flux_sigma, double* prod_mean,
                    double* prod_sigma, int64_t n_bins);

/* One generation's flux and production tallies per source particle (Sec. 2
   tallies, per generation). */
int mcx_get_generation_tallies(mcx_ctx* ctx, int32_t gen, double* flux, double* prod,
                               int64_t n_bins);

/* Per-history records of generation gen (record_histories = 1), n_per_gen
   entries indexed by history id.  Project addition, no passage (debug
   records for history-by-history parity). */
int mcx_get_records(mcx_ctx* ctx, int32_t gen, mcx_record* out, int64_t n);

/* Event log of generation gen: n = n_per_gen * event_log entries, history
   id major.  Project addition, no passage (debug). */
int mcx_get_event_log(mcx_ctx* ctx, int32_t gen, mcx_event* out, int64_t n);

/* Canonical fission bank of the last k-eigenvalue generation, ordered by
   (parent history, banking order): xyg[k][3] = x, y, group (energy in eV for
   continuous energy); *len receives
   the bank size (entries beyond cap are not written).  Paper Sec. 2: the
   fission bank of the event-based loop. */
int mcx_get_bank(mcx_ctx* ctx, double* xyg, int64_t cap, int64_t* len);

/* Timing of the last run (mcx_timing).  Project addition, no passage
   (Sec. 5 calls for profiling of the kernels). */
int mcx_get_timing(mcx_ctx* ctx, mcx_timing* out);

/* Load a batch of independent fixed-source problems (the batched form of
   the method: many problems of uneven size in one launch; project addition,
   no passage).  Every problem is
   validated as by mcx_load_geometry / mcx_load_mg_xs; all must share n_grp;
   1 <= n_probs <= 65535 and the total history count must stay below 2^32.
   Replaces any single problem loaded before (and vice versa); bind a
   workspace (mcx_workspace_size / mcx_bind_workspace with n_gen_max = 1)
   afterwards. */
int mcx_load_batch(mcx_ctx* ctx, int32_t n_probs, const mcx_problem* probs);

/* Run the loaded batch: one generation of every problem in one persistent
   launch, recorded once as a HIP graph (fill, transport, per-problem
   reduction) and replayed on ctx's stream.  Blocks until done.  Returns
   MCX_ELOST, MCX_EGUARD (results readable) or MCX_EDEVICE on failure.
   Project addition, no passage. */
int mcx_run_batch(mcx_ctx* ctx);

/* Per-problem results of the last batch, per source particle: k[p][3] =
   collision, track-length and absorption production estimators;
   counts[p][MCX_N_CNT].  Either may be NULL.  Project addition, no passage. */
int mcx_get_batch_results(mcx_ctx* ctx, double* k, int64_t* counts);

/* Flux and production tallies of problem p of the last batch, per source
   particle, in that problem's own bin order (as mcx_get_tallies);
   n_bins = nx * ny * (max_rings + 1) * n_grp of problem p.  Project addition,
   no passage. */
int mcx_get_batch_tallies(mcx_ctx* ctx, int32_t p, double* flux, double* prod, int64_t n_bins);

/* Pick the launch configuration with the shortest measured run of the bound
   problem or batch by timing a sweep of candidates on ctx's stream, and use
   it from then on: for the persistent engine and batches block, slots, grid,
   tau, then the collide-list ordering; for the event engine (multigroup or
   continuous energy) the block size, the flights per advance launch, the
   flights of the LDS-staged launches and the tail threshold, two
   generations per candidate.  A non-NULL
   cache_path names a text file of earlier results keyed by the workload's
   shape and the device: a hit skips the sweep, a miss appends the winner.
   Results do not depend on the configuration.  Overwrites the results of
   the last run.  Project addition, no passage. */
int mcx_autotune(mcx_ctx* ctx, const char* cache_path, mcx_tune* best);

/* Diagnostics of the device arithmetic (device pointers, on ctx's stream):
   which = 0: out[i] = ln(in[i]); 1: out[2i], out[2i+1] = cos, sin(2 pi in[i]);
   2: out[i] = sqrt(in[i]); 3: out[i] = uniform(bits of in[i]) mapping of a
   64-bit word to (0, 1).  Same functions the kernels call.  Project
   addition, no passage (diagnostics). */
int mcx_diag_math(mcx_ctx* ctx, int32_t which, const double* d_in, double* d_out, int64_t n);

/* The same functions evaluated on the host (no device needed).  Project
   addition, no passage (diagnostics). */
int mcx_host_math(int32_t which, const double* in, double* out, int64_t n);

/* Philox4x64-10 blocks on the device: in[i] = {c0, c1, c2, c3, k0, k1},
   out[i] = 4 output words (device pointers).  Paper Sec. 1 (replicable
   counter-based random numbers); diagnostics. */
int mcx_diag_philox(mcx_ctx* ctx, const uint64_t* d_in, uint64_t* d_out, int64_t n);

/* Message of the last failed call on ctx.  Project addition, no passage. */
const char* mcx_last_error(const mcx_ctx* ctx);

/* Release the context's host resources (never the caller's workspace).
   Project addition, no passage. */
void mcx_destroy(mcx_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
