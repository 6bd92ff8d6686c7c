/*
 * spkmc.h -- C ABI of the MI355X (gfx950) spkMC library.
 *
 * The library runs the synchronous parallel kinetic Monte Carlo cycle of
 * Martinez, Monasterio and Marian (arXiv:1005.4713) on a periodic L^3 Ising
 * lattice: Sec. 3.1 steps 1-6 with the sublattice steps 4a/4b of Sec. 3.2, the
 * energy of eq. 1 and the Glauber rates of eq. 3.  Every step of the cycle runs
 * in HIP kernels on the GPU; this header exposes plain C types only (no C++,
 * no torch, no exceptions) so that any caller can drive it.
 *
 * Conventions shared by all entry points
 *   - Lattice: N = L^3 sites, site (x, y, z) has linear index x + L (y + L z),
 *     periodic boundaries, neighbours counted with multiplicity (at L = 2 the
 *     +x and -x neighbour coincide and count twice).
 *   - Domains: edge d (even, d >= 2, L % d == 0), K = (L/d)^3 domains numbered
 *     kx + (L/d) (ky + (L/d) kz).  Each domain is split into 8 octants of edge
 *     h = d/2 (the 8-colour chessboard of Sec. 3.2, Fig. 1); colour s in 0..7
 *     has (sx, sy, sz) = (s & 1, (s >> 1) & 1, (s >> 2) & 1).  Same-colour
 *     octants are at least h sites apart, so they never interact.
 *   - Classes: class c = 7 [s_i = +1] + a_i, a_i = number of the 6 neighbours
 *     aligned with s_i; flip energy change dE_c = 2 J (2 a - 6) + 2 H s_i
 *     (eq. 1).  Rates (lambda = 1): Glauber r_c = 1 / (1 + exp(beta dE_c))
 *     (eq. 3 in its detailed-balance form), Metropolis r_c = min(1, exp(-beta dE_c)).
 *   - One cycle n (Sec. 3.1 / 3.2):
 *       4a. colour s_n = w0 >> 29 of Philox(ctr = (n_lo, n_hi, ~0, ~0), key = seed);
 *       1.  R_k = sum_{c=0..13} n_{k,c} r_c over the active octant (k, s_n),
 *           accumulated in class order with separate FP64 multiply and add;
 *       2.  R_max = max_k R_k (exact);
 *       3/4/4b. per domain, u = u53(w0, w1), w = w2 of Philox((n_lo, n_hi, k, s_n));
 *           target = u R_max; the first class c with target < running sum is
 *           chosen, none (target >= R_k) is the null event; the flipped site is
 *           the j-th (j = (w n_c) >> 32) site of class c in canonical order
 *           q = lx + h (ly + h lz) inside the octant;
 *       5.  t += -ln(u_t) / (8 R_max), u_t = uopen52(w2, w3) of the cycle draw
 *           (the 8 makes every spin flip at its physical rate);
 *       6.  flips become visible to every domain before the next cycle.
 *     u53(a, b) = ((a >> 5) 2^26 + (b >> 6)) / 2^53;
 *     uopen52(a, b) = ((((a >> 6) << 26) | (b >> 6)) + 1/2) / 2^52.
 *   - Initial spins (init = SPKMC_INIT_RANDOM): spin i is bit (i & 31) of word
 *     ((i >> 5) & 3) of Philox((b_lo, b_hi, 0xFFFFFFFE, 0xFFFFFFFE)), b = i >> 7;
 *     1 means +1.
 *   - Memory: the caller owns the device buffer (dev_buf, at least
 *     spkmc_state_bytes() bytes, 256-byte aligned, on the current HIP device)
 *     and the HIP stream; the library owns only the host-side context.  No
 *     entry point allocates device memory after spkmc_init.
 *   - Asynchrony: spkmc_init and spkmc_run only enqueue work on the stream;
 *     the other entry points that read device state synchronise the stream.
 *   - Errors: every call returns a status; spkmc_last_error() explains the
 *     last failure.  Nothing aborts the process.  A context whose device work
 *     failed answers SPKMC_E_STATE until destroyed.
 *   - Threading: one context per stream; calls on one context must not overlap.
 */
#ifndef SPKMC_H
#define SPKMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spkmc_ctx spkmc_ctx;

typedef enum spkmc_status {
    SPKMC_OK = 0,
    SPKMC_E_INVAL = 1,       /* invalid parameters or arguments                       */
    SPKMC_E_NOMEM = 2,       /* host allocation failed                                 */
    SPKMC_E_DEVICE = 3,      /* a HIP call or a kernel failed                          */
    SPKMC_E_STATE = 4,       /* context is in a failed state                           */
    SPKMC_E_RANGE = 5,       /* a buffer is too small                                  */
    SPKMC_E_UNSUPPORTED = 6  /* the requested engine does not support these parameters */
} spkmc_status;

enum { SPKMC_RATES_GLAUBER = 0, SPKMC_RATES_METROPOLIS = 1 };
enum { SPKMC_INIT_RANDOM = 0, SPKMC_INIT_UP = 1, SPKMC_INIT_DOWN = 2 };
/* Spin storage in the device buffer.  INT8: one byte per site, index x + L (y + L z).
 * PACKED: one bit per site, octant-major (domain k, colour s, canonical q), plus
 * every octant's own copy of its halo (the 6 layers of the octants that touch it);
 * needs h % 4 == 0. */
enum { SPKMC_LAYOUT_INT8 = 0, SPKMC_LAYOUT_PACKED = 1 };
/* Kernel engine.  AUTO picks PERSISTENT when supported (and when the domains
 * fit in one resident launch), else CYCLE.
 * CYCLE: three launches per cycle (bin, select-and-flip, finalize), any layout
 * and size (the only engine for lattices of 2^34 sites or more).
 * PERSISTENT: one cooperative launch per spkmc_run call with a device-wide R_max
 * exchange every cycle (PACKED layout, h = 8 or 16); every cycle bins the
 * active octant of every domain afresh.  With h = 16 and more lines than one
 * round of passes holds (up to 131 072 lines, e.g. two colours at L = 1024), the
 * wide mode keeps only each line's moments from the bin and derives the class
 * planes again for the selection, once the true R_max is known.
 * INCREMENTAL: the persistent launch, but the class histograms of all octants
 * stay on chip and follow every flip (the flipped site and its six neighbours
 * change class); a cycle classifies its active octant only to locate the
 * selected site, while the R_max exchange is in flight.
 * SLAB: the persistent launch for octant edge 16 (domain 32), variants 0 and
 * RMAX_ALL: the class counts of every octant, split over its four slabs of four
 * z-planes, stay in device memory (state_bytes grows by 896 bytes per domain
 * for PACKED lattices with domain 32) and follow every flip; a cycle reads the
 * counts of its active octant (of every octant with RMAX_ALL) instead of
 * binning it, and classifies only the slab that holds the selected site.
 * All engines produce bit-identical trajectories. */
enum { SPKMC_ENGINE_AUTO = 0, SPKMC_ENGINE_CYCLE = 1, SPKMC_ENGINE_PERSISTENT = 2, SPKMC_ENGINE_INCREMENTAL = 3,
       SPKMC_ENGINE_SLAB = 4 };

/* Method variants (bit flags).
 * RMAX_ALL (Sec. 3.1 step 2 read literally): R_max is the maximum over every
 *   octant of every colour, not only the active ones.
 * TWO_COLOURS (Sec. 3.2, first-neighbour interactions): the octants are
 *   coloured by the parity of sx + sy + sz; a cycle activates the four octants
 *   of the drawn colour in every domain, each its own frequency line with its
 *   own random stream (counter (n, domain, octant)); the colour is the top bit
 *   of the cycle word and the clock step uses S = 2.
 * RMAX_BOUND (Sec. 3.2, the optimistic alternative): R_max is the fixed bound
 *   R'_max = n_k max_c r_c (n_k sites per line), so no maximum over lines is
 *   taken; more null events, the same dynamics.
 * RMAX_ALL and RMAX_BOUND exclude each other.  Engines: CYCLE runs every
 * variant; PERSISTENT runs every combination of TWO_COLOURS and RMAX_BOUND;
 * INCREMENTAL runs 0 and RMAX_ALL; SLAB runs 0 and RMAX_ALL with domain 32.
 * AUTO: RMAX_ALL on SLAB where it runs, else on INCREMENTAL; the others on
 * PERSISTENT where it runs, else on CYCLE. */
enum { SPKMC_VARIANT_RMAX_ALL = 1, SPKMC_VARIANT_TWO_COLOURS = 2, SPKMC_VARIANT_RMAX_BOUND = 4 };

typedef struct spkmc_params {
    uint32_t struct_size; /* sizeof(spkmc_params): ABI check                           */
    int32_t L;            /* lattice edge, >= 2                                        */
    int32_t domain;       /* domain edge d: even, >= 2, L % d == 0                     */
    int32_t rates;        /* SPKMC_RATES_*                                             */
    double J;             /* coupling (eq. 1)                                          */
    double H;             /* external field (eq. 1)                                    */
    double T;             /* temperature, k_B = 1, > 0                                 */
    uint64_t seed;        /* Philox key (lo, hi)                                       */
    int32_t init;         /* SPKMC_INIT_*                                              */
    int32_t layout;       /* SPKMC_LAYOUT_*                                            */
    int32_t engine;       /* SPKMC_ENGINE_*                                            */
    int32_t wg_domains;   /* PERSISTENT: frequency lines per workgroup, 0 = default
                             (the fewest that fit the device at once); the row count
                             (32 for octant edge 16, 64 for 8) times 1, 2 or 4 passes,
                             for edge 16 also times 8 or 16 (the wide mode: two or
                             four rounds of four passes); INCREMENTAL: 32 rows times
                             1 or 2 passes.  Other values change the launch shape,
                             never the results                                      */
    uint32_t record_cap;  /* observation records kept on the device (ring)             */
    uint32_t variant;     /* SPKMC_VARIANT_* bits; 0 = 8 colours, R_max over the K
                             active octants                                          */
} spkmc_params;

/* One observation: the state after `cycle` cycles. */
typedef struct spkmc_record {
    uint64_t cycle;  /* cycles done                                      */
    uint64_t fired;  /* non-null events so far                           */
    uint64_t nulls;  /* null events so far (fired + nulls = K cycle)     */
    double t;        /* simulated time, units of 1/lambda                */
    int64_t M;       /* sum_i s_i (eq. 4 times N)                        */
    int64_t B;       /* sum_i sum_{e = x, y, z} s_i s_{i+e}              */
} spkmc_record;

typedef struct spkmc_obs {
    spkmc_record rec; /* current state                                   */
    double E;         /* -J B - H M (eq. 1)                              */
    double m;         /* M / N (eq. 4)                                   */
    double ur;        /* fired / (fired + nulls): utilisation (eq. 8)    */
} spkmc_obs;

typedef struct spkmc_info {
    int32_t engine;          /* engine in use (SPKMC_ENGINE_CYCLE or _PERSISTENT) */
    int32_t layout;          /* layout in use                                    */
    int32_t h;               /* octant edge                                      */
    int32_t grid;            /* workgroups of the cycle kernel(s)                */
    int32_t block;           /* threads per workgroup                            */
    int32_t wg_domains;      /* domains per workgroup (PERSISTENT)               */
    uint64_t K;              /* number of domains                                */
    uint64_t N;              /* number of sites                                  */
    uint64_t state_bytes;    /* bytes of device state                            */
    double bytes_per_cycle;  /* algorithmic bytes per cycle: K l ((h^3 + 6 h^2)/8 + 8)
                                with l active octants per domain (1; 4 with
                                TWO_COLOURS), plus K 2 x 112 for the slab engine's
                                count words                                       */
} spkmc_info;

/* Device bytes needed for these parameters; 0 if the parameters are invalid. */
size_t spkmc_state_bytes(const spkmc_params *p);

/* Validate p, compute the FP64 rate table on the host, lay out dev_buf and
 * enqueue the initial state on `hip_stream` (a hipStream_t; NULL = null stream).
 * *out receives the context (also on some errors, so spkmc_last_error can be
 * read; destroy it either way).
 * Errors: E_INVAL (bad parameters: d odd, d < 2, L % d != 0, L > 4096, T <= 0,
 * a rate that is 0 or not finite, unknown enum, wrong struct_size, unknown
 * variant bits or RMAX_ALL with RMAX_BOUND, PACKED with h % 4 != 0, 2^31 or
 * more frequency lines: (L/d)^3 domains, times 4 with TWO_COLOURS), E_RANGE
 * (dev_bytes too small), E_UNSUPPORTED
 * (engine PERSISTENT with parameters it cannot run), E_DEVICE. */
spkmc_status spkmc_init(const spkmc_params *p, void *dev_buf, size_t dev_bytes, void *hip_stream,
                        spkmc_ctx **out);

/* Enqueue `ncycles` cycles of the synchronous method (Sec. 3.1 steps 1-6, with
 * the sublattice steps 4a/4b of Sec. 3.2).  Every obs_every cycles (counted by the absolute
 * cycle number; 0 = never) a record of the state after that cycle is appended
 * to the device ring of record_cap entries. */
spkmc_status spkmc_run(spkmc_ctx *ctx, uint64_t ncycles, uint32_t obs_every);

/* Synchronise the stream and return the current state: counters, clock (Sec. 3.1
 * step 5), M and B, the energy of eq. 1, m of eq. 4 and the utilisation of eq. 8. */
spkmc_status spkmc_observables(spkmc_ctx *ctx, spkmc_obs *out);

/* Synchronise and copy the most recent min(cap, recorded, record_cap) records,
 * oldest first, to host memory; *n receives the number copied. */
spkmc_status spkmc_records(spkmc_ctx *ctx, spkmc_record *host, size_t cap, size_t *n);

/* Synchronise and copy all N spins (+1 / -1, index x + L (y + L z)) to host. */
spkmc_status spkmc_copy_spins(spkmc_ctx *ctx, int8_t *host, size_t n);

/* Replace all N spins from host memory (values +1 / -1) and recompute M and B;
 * counters, clock and cycle number are kept.  Synchronises. */
spkmc_status spkmc_set_spins(spkmc_ctx *ctx, const int8_t *host, size_t n);

/* The 14 FP64 rates c = 0..13 the library uses for these parameters (eq. 3 in its
 * detailed-balance form, or Metropolis; flip energies from eq. 1). */
spkmc_status spkmc_rate_table(const spkmc_params *p, double out[14]);

/* Checkpoint: with host == NULL, *n receives the blob size.  Otherwise the
 * state (parameters, counters, clock, records, spins) is copied to host
 * (cap bytes available).  Synchronises. */
spkmc_status spkmc_save(spkmc_ctx *ctx, void *host, size_t cap, size_t *n);

/* Restore a blob written by spkmc_save for the same parameters.  Resuming is
 * exact: the random streams are counter-based and keyed by the cycle number. */
spkmc_status spkmc_load(spkmc_ctx *ctx, const void *host, size_t n);

/* Launch shape and sizes of a context. */
spkmc_status spkmc_query(const spkmc_ctx *ctx, spkmc_info *out);

/* ------------------------------------------------------------------------- */
/* Batches: many independent lattices in one persistent launch.               */
/* ------------------------------------------------------------------------- */
typedef struct spkmc_batch_info {
    int32_t grid;        /* workgroups of the launch                               */
    int32_t block;       /* threads per workgroup                                  */
    int32_t wg_domains;  /* domains per workgroup                                  */
    int32_t h;           /* octant edge shared by the lattices                     */
    uint64_t lattices;   /* lattices in the launch (those with ncycles > 0)         */
    uint64_t domains;    /* sum of their domain counts                             */
} spkmc_batch_info;

/* Device workspace bytes spkmc_run_batch needs for n lattices. */
size_t spkmc_batch_workspace_bytes(size_t n);

/* Run ncycles[i] cycles (0 = skip) on each of n contexts in one cooperative
 * launch on their common stream.  Each lattice runs the cycle of spkmc_run
 * (Sec. 3.1); running many lattices in one launch is a scheduling choice of this
 * library, not an operation of the method.  The lattices stay independent: each keeps its
 * own clock, R_max, random streams and records, and the result of every
 * lattice is bit-identical to running it alone with spkmc_run.  All contexts
 * must use the PACKED layout with the same octant edge (8 or 16) and the same
 * stream, each context at most once (E_INVAL otherwise; a context with
 * ncycles 0 is not counted), and the launch must fit on the device at once (E_UNSUPPORTED
 * otherwise: split the batch).  wg_domains: domains per workgroup (0 = the
 * fewest passes that fit; 1, 2 or 4 passes of the row count, at most 2 for
 * octant edge 8).  dev_workspace: spkmc_batch_workspace_bytes(n)
 * bytes of device memory owned by the caller; it must stay untouched until
 * the launch has finished.  info (may be NULL) receives the launch shape. */
spkmc_status spkmc_run_batch(spkmc_ctx *const *ctxs, size_t n, const uint64_t *ncycles, uint32_t obs_every,
                             int32_t wg_domains, void *dev_workspace, size_t ws_bytes, spkmc_batch_info *info);

/* spkmc_run_batch for callers that cannot allocate device memory (tight serving
 * loops, harnesses that forbid allocation): the same launch with the same
 * results, bit for bit, but the descriptors go into a device array of the
 * library (one per GPU, 512 descriptors, kept until the process ends) instead
 * of a caller's workspace.  It calls no hipMalloc or hipFree; its first call
 * on a device resolves that device's array address.  At most 512 lattices per
 * call (E_RANGE otherwise).  Every call on one GPU shares the array: calls
 * whose launches can overlap on one GPU (different streams) race and must not
 * be made; calls on one stream run in order.  Arguments and errors otherwise as
 * for spkmc_run_batch. */
spkmc_status spkmc_run_batch_static(spkmc_ctx *const *ctxs, size_t n, const uint64_t *ncycles, uint32_t obs_every,
                                    int32_t wg_domains, spkmc_batch_info *info);

/* A batch macro-step captured once into a HIP graph and replayed: the slot and
 * flag set-up, the persistent batch launch and a kernel that advances every
 * descriptor's start cycle by its cycle count, so that each replay continues
 * every lattice where the last one stopped, with no host work per replay.
 * Arguments as for spkmc_run_batch; dev_workspace (spkmc_batch_workspace_bytes(n)
 * bytes, caller-owned) holds the descriptors for the graph's whole life and
 * must stay untouched until the graph is destroyed and its last replay has
 * finished.  Nothing runs at creation but the descriptor upload.  While the
 * graph lives its members advance only through spkmc_batch_graph_launch
 * (E_STATE from there if a member's cycle count moved otherwise), and every
 * member context must outlive the graph (the graph keeps pointers to them;
 * destroying a member first leaves them dangling).  Replays are
 * bit-identical to spkmc_run_batch and to solo runs.  The batch kernel is a
 * cooperative graph node.  E_UNSUPPORTED if the runtime cannot build or
 * instantiate the graph. */
typedef struct spkmc_batch_graph spkmc_batch_graph;
spkmc_status spkmc_batch_graph_create(spkmc_ctx *const *ctxs, size_t n, const uint64_t *ncycles, uint32_t obs_every,
                                      int32_t wg_domains, void *dev_workspace, size_t ws_bytes,
                                      spkmc_batch_info *info, spkmc_batch_graph **out);
/* Enqueue `replays` replays of the macro-step on the members' stream (async). */
spkmc_status spkmc_batch_graph_launch(spkmc_batch_graph *graph, uint32_t replays);
/* Frees the graph (host side and the runtime's graph objects; not the workspace). */
void spkmc_batch_graph_destroy(spkmc_batch_graph *graph);

/* ------------------------------------------------------------------------- */
/* Serving: a request loop with continuous batching.                          */
/* ------------------------------------------------------------------------- */
/* Serving is a scheduling layer of this library, not an operation of the method:
 * every request runs the cycle of spkmc_run (Sec. 3.1).
 * A server owns a caller-provided device pool and a stream.  Requests (one
 * lattice each: spkmc_params, a cycle count and an observation interval) are
 * queued in FIFO order and admitted while a slot is free and their footprint
 * (spkmc_state_bytes, first fit in the pool) fits; the lattice and its clock
 * then stay resident in the pool until the request has run all its cycles.
 * All resident requests advance together in macro-steps of macro_cycles
 * cycles: per macro-step, PACKED lattices with an octant edge of 8 or 16 share
 * cooperative batch launches (one per edge, split only where the device cannot
 * hold them at once); the others run alone with spkmc_run.  Requests that
 * arrive while others run join at the next macro-step.  A macro-step is only
 * a scheduling unit: the random streams are keyed by each lattice's own cycle
 * number, so every request ends bit-identical to running it alone with
 * spkmc_init + spkmc_run (engine, wg_domains and the launch shape never change
 * results).  Times are seconds on the server's monotonic clock (0 = creation).
 *
 * Threading: a server and its requests are driven from one thread at a time.
 * The pool, the stream and the server's pinned host slots are used until
 * spkmc_server_destroy returns. */
typedef struct spkmc_server spkmc_server;

typedef struct spkmc_server_config {
    uint32_t struct_size;   /* sizeof(spkmc_server_config)                        */
    uint32_t macro_cycles;  /* cycles per macro-step, > 0                         */
    uint32_t max_live;      /* requests resident at once, 1..4096                 */
    uint32_t inflight;      /* macro-steps enqueued ahead of the device, 1..8     */
    int32_t wg_domains;     /* batch launches: domains per workgroup (0 = fewest
                               passes that fit); never changes results            */
    uint32_t reserved;      /* must be 0                                          */
} spkmc_server_config;

enum {
    SPKMC_REQ_QUEUED = 0,   /* waiting for a slot and pool memory                   */
    SPKMC_REQ_RUNNING = 1,  /* resident; macro-steps enqueued                       */
    SPKMC_REQ_DONE = 2,     /* all cycles finished on the device; obs valid         */
    SPKMC_REQ_FAILED = 3    /* rejected at admission or a launch failed (message in
                               spkmc_server_last_error at the time)                 */
};

/* submit flags */
enum { SPKMC_SERVE_KEEP = 1 }; /* keep the lattice resident after DONE, so that
                                  spkmc_server_context can be used to read spins
                                  and records, until spkmc_server_release      */

typedef struct spkmc_request_status {
    int32_t state;          /* SPKMC_REQ_*                                         */
    uint32_t flags;         /* as submitted                                        */
    uint64_t ncycles;       /* cycles requested                                    */
    uint64_t cycles_enqueued;
    uint64_t bytes;         /* pool footprint                                      */
    double t_arrival;       /* as submitted (or the submit time)                   */
    double t_admit;         /* admission (-1 while queued)                         */
    double t_done;          /* first time step() saw the last macro-step finished  */
    spkmc_obs obs;          /* final state when DONE                               */
} spkmc_request_status;

typedef struct spkmc_server_stats {
    uint64_t queued, live, finishing, done, failed; /* requests by state; finishing =
                                                       last macro-step enqueued, not
                                                       yet seen finished            */
    uint64_t macro_steps;     /* macro-steps enqueued                               */
    uint64_t launches;        /* batch launches + solo runs enqueued                */
    uint64_t pool_in_use;     /* bytes of the pool held by resident requests        */
    uint64_t pool_peak;       /* high-water mark of pool_in_use                     */
    uint64_t inflight;        /* macro-steps enqueued and not yet seen finished     */
} spkmc_server_stats;

/* Bytes of the pool the server reserves for itself (batch descriptors) for this
 * configuration; 0 if the configuration is invalid.  The rest holds lattices. */
size_t spkmc_server_reserved_bytes(const spkmc_server_config *cfg);

/* Create a server over dev_pool (pool_bytes of device memory owned by the
 * caller; 256-byte aligned) and hip_stream (a hipStream_t; NULL = null stream).
 * Allocates host memory and max_live * (inflight + 1) pinned 256-byte slots.
 * Errors: E_INVAL (bad configuration or pool), E_RANGE (pool smaller than the
 * reserved bytes), E_NOMEM, E_DEVICE. */
spkmc_status spkmc_server_create(const spkmc_server_config *cfg, void *dev_pool, size_t pool_bytes,
                                 void *hip_stream, spkmc_server **out);

/* Queue a request; *id receives its id (ids start at 1 and are never reused).
 * t_arrival < 0 means now.  obs_every as in spkmc_run.  The parameters are
 * validated at once (E_INVAL as spkmc_init; E_RANGE if the footprint exceeds
 * what the pool can ever hold). */
spkmc_status spkmc_server_submit(spkmc_server *s, const spkmc_params *p, uint64_t ncycles, uint32_t obs_every,
                                 uint32_t flags, double t_arrival, uint64_t *id);

/* Make progress without blocking the device: retire macro-steps the device has
 * finished (their finishing requests become DONE), admit queued requests, and
 * enqueue macro-steps until `inflight` are outstanding.  With wait != 0 and
 * nothing retired, first block until the oldest outstanding macro-step has
 * finished.  stats (may be NULL) receives the counts after the call. */
spkmc_status spkmc_server_step(spkmc_server *s, int wait, spkmc_server_stats *stats);

/* Status of a request (E_INVAL for an unknown or released id). */
spkmc_status spkmc_server_poll(const spkmc_server *s, uint64_t id, spkmc_request_status *out);

/* The context of a DONE request submitted with SPKMC_SERVE_KEEP, for
 * spkmc_copy_spins / spkmc_records / spkmc_observables / spkmc_save.  It stays
 * owned by the server and is valid until spkmc_server_release. */
spkmc_status spkmc_server_context(spkmc_server *s, uint64_t id, spkmc_ctx **ctx);

/* Forget a DONE or FAILED request and free what it still holds (the lattice
 * of a kept request).  E_STATE while it is queued or running. */
spkmc_status spkmc_server_release(spkmc_server *s, uint64_t id);

/* Seconds since the server was created (its clock). */
double spkmc_server_clock(const spkmc_server *s);

/* Message of the last failure of a call on s (s == NULL: as spkmc_last_error(NULL)). */
const char *spkmc_server_last_error(const spkmc_server *s);

/* Synchronise the stream, then free the server, its contexts and pinned slots
 * (not the pool or the stream). */
void spkmc_server_destroy(spkmc_server *s);

/* Message of the last failure on ctx (ctx == NULL: of the last failed call
 * that had no context on this thread).  Never NULL. */
const char *spkmc_last_error(const spkmc_ctx *ctx);

/* Free the host context.  Does not free dev_buf or the stream. */
void spkmc_destroy(spkmc_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SPKMC_H */
