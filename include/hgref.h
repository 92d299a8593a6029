/*
 * hgref.h -- C ABI of the MI355X (gfx950) km1 label-propagation refinement
 * core: pin counts, connectivity, km1, k-way move gains and synchronous,
 * deterministic label-propagation rounds on a hypergraph.
 *
 * Paper: Gottesbueren, Heuer, Sanders, Schlag, "Scalable Shared-Memory
 * Hypergraph Partitioning" (arXiv 2010.10272).  The operations follow its
 * problem statement (section "Preliminaries"), its gain definitions (section
 * "Parallel Gain Calculation", subsections "Data Structures for Gain
 * Calculation" and "Attributed Gains") and its label-propagation refinement
 * (section "Label Propagation"), re-specified as synchronous rounds.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All arrays are DEVICE memory owned by the caller (for example PyTorch
 *   tensors).  The library never allocates or frees device memory; scratch
 *   space comes from the caller's workspace (hg_workspace_size).  Buffers
 *   must stay alive until the work queued on `stream` has completed and, for
 *   the arrays a graph handle borrows, until hg_free.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *   only enqueue work and return, except hg_load_csr and hg_sync_status,
 *   which synchronize the stream.
 * - Integers only.  Vertex ids, net ids, block ids, vertex and net weights and
 *   pin counts are int32; offsets, block weights, gains and km1 are int64.
 *   Blocks are numbered 0..k-1 (the paper numbers them 1..k).
 * - Supported sizes: 1 <= n, m < 2^31; m <= P < 2^31 pins; 2 <= k <= 256;
 *   positive weights; total net weight sum_e w(e) < 2^31 and total vertex
 *   weight < 2^62.  Larger values return HG_ERR_UNSUPPORTED.
 * - Errors: every call returns an hg_status.  Host-side argument checks run
 *   before anything is enqueued; on failure nothing is enqueued and
 *   hg_last_error() describes the problem.  Values read from device arrays
 *   (partition ids) are checked on the device: an out-of-range value is
 *   skipped, never used as an index, and raises a flag that hg_sync_status
 *   reports.  A device fault surfaces as HG_ERR_DEVICE at the next call that
 *   synchronizes.
 * - Results are deterministic: the same inputs give bit-identical outputs,
 *   whatever the order in which the GPU runs its work items.
 */
#ifndef HGREF_H
#define HGREF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hg_status;
#define HG_OK 0
#define HG_ERR_INVALID (-1)      /* malformed input (null pointer, bad CSR, ...) */
#define HG_ERR_UNSUPPORTED (-2)  /* valid but outside the supported sizes        */
#define HG_ERR_DEVICE (-3)       /* a HIP runtime call failed                    */
#define HG_ERR_WORKSPACE (-4)    /* workspace too small for this n, m, P or k    */

#define HG_MAX_K 256

/* Opaque host object describing one loaded hypergraph.  It borrows the
 * caller's device arrays (net CSR, weights, incidence CSR, workspace) and
 * holds a few host-side facts about them (sizes, total weights, degree
 * classes).  Not thread-safe: one handle is used by one host thread. */
typedef struct hg_graph_s* hg_graph;

/* One record per label-propagation round, written to DEVICE memory.
 * Counts refer to the round-start state S_r (section "Label Propagation"). */
typedef struct {
  int64_t eligible;              /* vertices eligible in this round                 */
  int64_t boundary;              /* eligible vertices incident to a cut net         */
  int64_t candidates;            /* vertices whose best move passes the move rule   */
  int64_t approved;              /* moves approved against L_max and applied        */
  int64_t moved_pins;            /* sum of d(u) over moved vertices                 */
  int64_t touched_nets;          /* nets holding at least one moved vertex          */
  int64_t km1_delta;             /* attributed km1 reduction of the round           */
  int64_t km1_after;             /* km1 after the round                             */
  int64_t max_block_weight;      /* max_i c(V_i) after the round                    */
  int64_t km1_delta_recomputed;  /* sum over touched nets of (lambda_old -
                                    lambda_new) * w(e); equals km1_delta           */
  int64_t active_pins;           /* sum of d(u) over active (eligible boundary) u   */
  int64_t touched_pins;          /* sum of |e| over touched nets (pins made eligible,
                                    counted with repeats)                          */
} hg_round_stats;

/* Phases of a label-propagation round measured by hg_timing_collect. */
#define HG_PHASE_SELECT 0    /* select sweep (light and heavy vertices)            */
#define HG_PHASE_APPROVE 1   /* thresholds, tile sums and scan, approve + apply     */
#define HG_PHASE_FINALIZE 2  /* touched-net finalize and the round record          */
#define HG_NUM_PHASES 3

/* Static facts about a loaded hypergraph (host memory). */
typedef struct {
  int32_t n, m;
  int64_t P;
  int64_t total_vertex_weight;   /* c(V)                                            */
  int64_t total_net_weight;      /* w(E)                                            */
  int32_t max_degree;            /* max_v d(v)                                      */
  int32_t max_net_size;          /* max_e |e|                                       */
  int32_t max_incident_weight;   /* max_v w(I(v)), an upper bound of every gain     */
  int32_t heavy_vertices;        /* vertices with w(I(v)) > 255 (wavefront path)    */
} hg_graph_info;

/* Number of 32-bit words per net in the net-state array for a given k:
 * 2 + 2*ceil(k/32) rounded up to a power of two (4, 8, 16 or 32).  Returns 0
 * for an unsupported k.
 *
 * Net-state layout: uint32 netstate[hg_netstate_words(m, k)].  The first
 * m * hg_net_words(k) words hold one record per net (row e):
 *   word 0                 w(e), the net weight (copied at pin-count time)
 *   word 1                 lambda(e) = |Lambda(e)|
 *   words 2 .. 2+W-1       Lambda(e) as a bitset: bit i%32 of word 2+i/32 is
 *                          set iff Phi(e,i) > 0  (W = ceil(k/32) rounded up
 *                          to 1, 2, 4 or 8)
 *   words 2+W .. 2+2W-1    S(e): bit i set iff Phi(e,i) == 1 (blocks holding
 *                          exactly one pin of e; b(u) needs only this)
 *   remaining words        zero
 * For k <= 64 a compact copy of the two bitsets follows the records, V words
 * per net (V = 1 for k <= 16: Lambda in bits 0-15, S in bits 16-31; V = 2 for
 * k <= 32: Lambda, S; V = 4 for k <= 64: Lambda lo, hi, S lo, hi).  It is
 * kept up to date only when every net weight is 1, and then the gain sweeps
 * read it instead of the full records.  Callers treat it as opaque.
 * The paper keeps Phi(e,i) and Lambda(e) per net in its partition data
 * structure (subsection "Data Structures for Gain Calculation"); this packs
 * what a gain computation reads for one net into one aligned record. */
int32_t hg_net_words(int32_t k);

/* Total 32-bit words of a net-state array for m nets and k blocks (records
 * plus the compact copy described above); 0 for unsupported arguments. */
int64_t hg_netstate_words(int32_t m, int32_t k);

/* Bytes of device workspace needed for a hypergraph with n vertices, m nets
 * and P pins, refined with any k <= k_max.  0 if the sizes are unsupported. */
size_t hg_workspace_size(int32_t n, int32_t m, int64_t P, int32_t k_max);

/* Load a hypergraph given as net CSR and build its incidence CSR
 * (section "Preliminaries": nets are vertex sets, I(v) the incident nets).
 *   eptr   int64[m+1]   offsets into pins; eptr[0] = 0, eptr[m] = P
 *   pins   int32[P]     pins of net e at pins[eptr[e] .. eptr[e+1])
 *   vwgt   int32[n]     vertex weights c(v) > 0, or NULL for unit weights
 *   ewgt   int32[m]     net weights w(e) > 0, or NULL for unit weights
 *   vptr   int64[n+1]   OUT: incidence offsets
 *   vnets  int32[P]     OUT: I(v) at vnets[vptr[v] .. vptr[v+1]), increasing
 *   workspace, ws_bytes caller scratch of at least
 *                       hg_workspace_size(n, m, P, k_max) bytes
 *   k_max               largest k later calls will use (2..256)
 * Checks (on the device, always): eptr increasing with eptr[0] = 0 and
 * eptr[m] = P (no empty net), pins in [0,n), no vertex twice in a net,
 * weights > 0, total net weight < 2^31.  Single-pin nets are allowed.
 * Synchronizes `stream` (twice) and returns HG_ERR_INVALID or
 * HG_ERR_UNSUPPORTED on bad input, with *out left NULL.  The handle borrows
 * eptr, pins, vwgt, ewgt, vptr, vnets and workspace. */
hg_status hg_load_csr(int32_t n, int32_t m, int64_t P, const int64_t* eptr,
                      const int32_t* pins, const int32_t* vwgt, const int32_t* ewgt,
                      int64_t* vptr, int32_t* vnets, void* workspace, size_t ws_bytes,
                      int32_t k_max, void* stream, hg_graph* out);

/* Release the host handle (device arrays stay with the caller). */
void hg_free(hg_graph g);

/* Copy the static facts gathered by hg_load_csr into *info. */
hg_status hg_get_info(hg_graph g, hg_graph_info* info);

/* L_max = (1 + eps) * ceil(c(V) / k) (section "Preliminaries"), as the
 * integer floor((1 + eps) * ceil(c(V)/k)) computed in IEEE double; block
 * weights are integers, so c(V_i) <= L_max is the same test.  Requires
 * 0 < eps < 1.  Returns -1 on bad arguments. */
int64_t hg_max_block_weight(hg_graph g, int32_t k, double eps);

/* Pin counts Phi(e,i), connectivity sets and block weights from a partition
 * (section "Preliminaries").
 *   part      int32[n]        block of every vertex, in [0,k)
 *   phi       int32[m*k]      OUT: Phi(e,i) at phi[e*k + i]
 *   netstate  uint32[m*hg_net_words(k)]  OUT: per-net record (see above)
 *   block_w   int64[k]        OUT: c(V_i)
 *   km1_out   int64[1] or NULL OUT: sum_e (lambda(e) - 1) w(e)
 * Each net is counted by one group of lanes, so no atomics touch Phi. */
hg_status hg_compute_pincounts(hg_graph g, int32_t k, const int32_t* part, int32_t* phi,
                               uint32_t* netstate, int64_t* block_w, int64_t* km1_out,
                               void* stream);

/* Connectivity metric km1 = sum_e (lambda(e) - 1) w(e) (section
 * "Preliminaries") from a net-state array; int64 result in km1_out[0]. */
hg_status hg_km1(hg_graph g, int32_t k, const uint32_t* netstate, int64_t* km1_out,
                 void* stream);

/* All k-way move gains (section "Parallel Gain Calculation"):
 *   b(u)   = w({e in I(u) : Phi(e, Pi(u)) = 1})
 *   p_i(u) = w({e in I(u) : Phi(e, i) = 0})
 *   gains[u*k + i] = b(u) - p_i(u) for i != Pi(u), and 0 for i = Pi(u)
 *   gains is int64[n*k], row-major (vertex-major), 16-byte aligned
 *   (HG_ERR_INVALID otherwise)
 *   benefit[u] = b(u) (int64[n], may be NULL)
 * part and netstate must describe the same partition (hg_compute_pincounts
 * or a sequence of hg_lp_round calls establishes that).  Rows are written
 * with streaming (nontemporal) stores. */
hg_status hg_gains(hg_graph g, int32_t k, const int32_t* part, const uint32_t* netstate,
                   int64_t* gains, int64_t* benefit, void* stream);

/* One synchronous label-propagation round (section "Label Propagation",
 * re-specified as select / approve / apply on the round-start state):
 *  1. eligible vertices (eligible[v] != 0) that touch a cut net are active;
 *  2. each active u picks, among neighbouring blocks i (some net of I(u) has
 *     a pin in i) with c(V_i) + c(u) <= max_block_w, the best by (gain desc,
 *     c(V_i) asc, i asc); it is a candidate if that gain is > 0, or 0 with
 *     c(V_t) + c(u) < c(V_Pi(u));
 *  3. per target block t, candidates in (gain desc, vertex id asc) order are
 *     approved as the longest prefix with c(V_t) + prefix weight <= L_max;
 *  4. approved moves are applied at once: part, phi (integer atomics),
 *     netstate of every touched net and block_w are updated, *km1 drops by
 *     the attributed gain (subsection "Attributed Gains");
 *  5. eligible is rewritten to mark every pin of every net holding a moved
 *     vertex (the movers and their neighbours), and moved[v] = 1 for movers.
 *   part, phi, netstate, block_w  in/out state of one partition (consistent)
 *   eligible uint8[n]     in/out; set all to 1 before the first round
 *   moved    uint8[n]     OUT, or NULL
 *   km1      int64[1]     in/out: km1 of the state before/after the round
 *   stats    hg_round_stats[1]  OUT (device)
 * max_block_w is L_max (hg_max_block_weight). */
hg_status hg_lp_round(hg_graph g, int32_t k, int64_t max_block_w, int32_t* part,
                      int32_t* phi, uint32_t* netstate, int64_t* block_w,
                      uint8_t* eligible, uint8_t* moved, int64_t* km1,
                      hg_round_stats* stats, void* stream);

/* hg_lp_round for callers that cannot allocate device memory at call time
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as hg_lp_round; the round
 * scratch (candidate words, touched-net flags, gain histograms, thresholds,
 * tile sums, counter and block-weight slots) comes from a fixed device array
 * inside the library (about 15 MB, one copy per GPU, held until the process
 * ends) instead of the graph's workspace, and the call allocates nothing.
 * Limits: n <= 2^20 and m <= 2^20 (HG_ERR_UNSUPPORTED beyond, nothing
 * enqueued); any k the graph supports.  `stream` must belong to the current
 * device.  Every call on one GPU shares that GPU's array and clears what
 * must start at zero (with fill kernels, no memset nodes), so calls whose
 * work overlaps on one GPU (other streams or host threads) race and give
 * undefined results; calls on one stream are ordered and safe.  Per-phase
 * timing (hg_timing_enable) does not apply to this call. */
hg_status hg_lp_round_noalloc(hg_graph g, int32_t k, int64_t max_block_w, int32_t* part,
                              int32_t* phi, uint32_t* netstate, int64_t* block_w,
                              uint8_t* eligible, uint8_t* moved, int64_t* km1,
                              hg_round_stats* stats, void* stream);

/* Refinement driver: hg_compute_pincounts from `part`, every vertex
 * eligible, then `rounds` label-propagation rounds with
 * L_max = hg_max_block_weight(g, k, eps).  Rounds after convergence record
 * zero moves.  part is refined in place; phi, netstate, block_w and eligible
 * are caller buffers used as state and hold the final state on return;
 * stats[rounds] (device) receives one record per round; km1_out[0] (device)
 * the final km1.  use_graph != 0 records the rounds once into a hipGraph and
 * replays it (the record is kept in the handle and reused while the same
 * buffers, k and round count are passed). */
hg_status hg_refine(hg_graph g, int32_t k, double eps, int32_t rounds, int32_t* part,
                    int32_t* phi, uint32_t* netstate, int64_t* block_w, uint8_t* eligible,
                    hg_round_stats* stats, int64_t* km1_out, int32_t use_graph,
                    void* stream);

/* ------------------------------------------------------------------------
 * Gain cache (subsection "Gain Caching").  Instead of the k gains of every
 * vertex the cache keeps their two terms apart, so that a round's moves
 * change few entries:
 *   int32 cache[0 .. n)           b(u) = w({e in I(u) : Phi(e, Pi(u)) = 1})
 *   int32 cache[n .. 2n)          w(I(u))
 *   int32 cache[pb + u*ks + i]    p_i(u) = w({e in I(u) : Phi(e, i) = 0}),
 *                                 pb = 2n rounded up to a multiple of 4,
 *                                 ks = k rounded up to a multiple of 4
 * and g_i(u) = b(u) - p_i(u) for i != Pi(u).  The buffer is the caller's
 * (device, 16-byte aligned, hg_gain_cache_bytes bytes) and belongs to one
 * (graph, k, state) at a time.  A cached round makes the same decisions as
 * hg_lp_round on the same state (every output bit-identical) and leaves the
 * cache equal to the cache of the new partition: the finalize step applies
 * the paper's four update rules summed over the round's moves (for every pin
 * v of a net e that held a mover: p_i(v) -/+ w(e) where block i entered/left
 * Lambda(e); b(v) of a pin that did not move -/+ w(e) where its block
 * left/entered the set of blocks with exactly one pin of e), then b(u) is
 * recomputed for every moved vertex.  Entries padding a row are never read.
 * ------------------------------------------------------------------------ */

/* Bytes of the gain cache of n vertices at k blocks; -1 on bad arguments. */
int64_t hg_gain_cache_bytes(int32_t n, int32_t k);

/* Fill the cache from a partition and its net state (hg_compute_pincounts
 * or earlier rounds); same requirements as hg_gains. */
hg_status hg_gain_cache_init(hg_graph g, int32_t k, const int32_t* part, const uint32_t* netstate,
                             int32_t* cache, void* stream);

/* hg_lp_round reading the gains from `cache` and updating it.  `moved` is
 * required (the update reads it); `cache` must hold the cache of the current
 * partition (hg_gain_cache_init, or the previous cached round). */
hg_status hg_lp_round_cached(hg_graph g, int32_t k, int64_t max_block_w, int32_t* part,
                             int32_t* phi, uint32_t* netstate, int64_t* block_w,
                             uint8_t* eligible, uint8_t* moved, int64_t* km1,
                             hg_round_stats* stats, int32_t* cache, void* stream);

/* hg_refine (without a graph) through the cache: pin counts from part, every
 * vertex eligible, hg_gain_cache_init, then `rounds` cached rounds.  Outputs
 * are bit-identical to hg_refine. */
hg_status hg_refine_cached(hg_graph g, int32_t k, double eps, int32_t rounds, int32_t* part,
                           int32_t* phi, uint32_t* netstate, int64_t* block_w, uint8_t* eligible,
                           uint8_t* moved, hg_round_stats* stats, int64_t* km1_out,
                           int32_t* cache, void* stream);

/* Per-phase timing of label-propagation rounds, off by default.  While on,
 * every round enqueued outside a stream capture (hg_lp_round, and hg_refine
 * with use_graph = 0) records HIP events on its own stream around the three
 * phases (four per round; inside one refine call a round starts at the
 * previous round's end event, so three); a recorded hipGraph is never
 * timed. */
hg_status hg_timing_enable(hg_graph g, int32_t enable);

/* Wait for the recorded events, add each phase's total duration in
 * milliseconds to ms[HG_NUM_PHASES] and the number of timed rounds to
 * *rounds, then forget the events. */
hg_status hg_timing_collect(hg_graph g, double* ms, int64_t* rounds);

/* Synchronize `stream`, then report HG_ERR_INVALID if a device-side check
 * (a partition id outside [0,k)) fired since the last call, HG_ERR_DEVICE
 * if the stream reported an error, HG_OK otherwise.  Clears the flag. */
hg_status hg_sync_status(hg_graph g, void* stream);

/* Message for the last non-OK status returned on this host thread. */
const char* hg_last_error(void);

/* ------------------------------------------------------------------ batches
 * Many independent refinements advanced together.  Every kernel of a round
 * (and of the pin-count pass that starts a refinement) is launched once for
 * the whole batch; each workgroup reads its instance and its share of the
 * work from a table in caller device memory.  An instance's sweeps are
 * placed on one XCD (large instances: spread over all eight), so its net
 * records stay in that XCD's L2.  The arithmetic is that of the single-
 * instance calls: every output is bit-identical to hg_refine on the instance
 * alone, whatever else shares the batch. */

typedef struct hg_batch_s* hg_batch;

/* One member of a batch: a loaded hypergraph and the caller's state for one
 * k-way partition of it (the buffers hg_refine takes, same layouts).  A graph
 * handle may appear in at most one member of a batch, and in at most one
 * batch (or hg_* call) whose work is in flight: its workspace is the
 * refinement's scratch space. */
typedef struct {
  hg_graph g;
  int32_t k;                 /* 2 <= k <= k_max of g                            */
  int32_t reserved;          /* set to 0                                         */
  double eps;                /* L_max = hg_max_block_weight(g, k, eps)           */
  int32_t* part;             /* int32[n] in/out                                  */
  int32_t* phi;              /* int32[m*k]                                       */
  uint32_t* netstate;        /* uint32[hg_netstate_words(m, k)]                  */
  int64_t* block_w;          /* int64[k]                                         */
  uint8_t* eligible;         /* uint8[n]                                         */
  hg_round_stats* stats;     /* round r of hg_batch_round writes stats[r]        */
  int64_t* km1;              /* int64[1]: km1 of the current state               */
} hg_instance;

/* How the batched sweeps split one instance's work into workgroups, for the
 * instances of one size class.  Any schedule gives the same results; only the
 * speed differs (hg_batch_autotune measures). */
typedef struct {
  int32_t select_chunks;     /* 256-vertex chunks per select workgroup, 1..64    */
  int32_t finalize_chunks;   /* 1024-net blocks per finalize workgroup, 1..64    */
  int32_t count_chunks;      /* 256-net chunks per pin-count workgroup, 1..64    */
  int32_t net_lanes;         /* lanes per net in the pin-count and finalize
                                sweeps: 0 = the minimum for k (4 for k <= 4, 8
                                for k <= 64, 16 for k <= 128, else 32), or 4, 8,
                                16, 32 (raised to that minimum)                  */
} hg_schedule;

/* Size classes, by vertex count n: [0, 2^13), [2^13, 2^16), [2^16, 2^19),
 * [2^19, 2^31).  A schedule argument is an array of HG_SIZE_CLASSES entries;
 * NULL means the built-in defaults. */
#define HG_SIZE_CLASSES 4

/* Device bytes of the work table for these members: enough for every
 * schedule (so hg_batch_autotune can use the same table).  0 on bad input. */
size_t hg_batch_table_bytes(const hg_instance* members, int32_t count);

/* Check the members (as hg_refine checks its arguments, plus: no graph
 * twice), place them on XCDs, build the work tables for `sched` and copy
 * them to `table` (device, table_bytes >= hg_batch_table_bytes) on `stream`.
 * The handle keeps a host copy of the members; `table` must stay alive until
 * hg_batch_free.  Members are numbered 0..count-1 in the given order. */
hg_status hg_batch_create(const hg_instance* members, int32_t count, const hg_schedule* sched,
                          void* table, size_t table_bytes, void* stream, hg_batch* out);

/* Release the handle (waits for its last table copy; device arrays stay). */
void hg_batch_free(hg_batch b);

/* Start every member's refinement: pin counts, net state, block weights and
 * km1 from its partition, every vertex eligible (hg_compute_pincounts plus
 * the set-up hg_refine does). */
hg_status hg_batch_start(hg_batch b, void* stream);

/* One label-propagation round (as hg_lp_round with L_max from eps and no
 * moved flags) for every member; member i's record goes to stats_i[round]. */
hg_status hg_batch_round(hg_batch b, int32_t round, void* stream);

/* hg_batch_start, then rounds 0..rounds-1.  use_graph != 0 records the whole
 * sequence once into one hipGraph (kept in the handle while `rounds` stays
 * the same) and launches it. */
hg_status hg_batch_refine(hg_batch b, int32_t rounds, int32_t use_graph, void* stream);

/* Measure schedules and keep the fastest per size class.  For each class
 * present, each field of the schedule in turn takes each of its candidate
 * values (chunks 1, 2, 4, 8, 16; lanes 0, 2x minimum); a trial runs
 * hg_batch_start and one round on the members of that class, `repeats` times
 * (best time wins).  The members' partitions are saved into part_save
 * (device int32, at least the sum of their n) first and restored after every
 * trial, so on return each member's `part` is unchanged and its other state
 * must be rebuilt (hg_batch_start).  Synchronizes `stream`.  The chosen
 * schedules are written to best[HG_SIZE_CLASSES] (may be NULL) and the
 * batch's tables are rebuilt with them. */
hg_status hg_batch_autotune(hg_batch b, int32_t* part_save, int64_t save_elems,
                            int32_t repeats, void* stream, hg_schedule* best);

/* The batch's current schedules (HG_SIZE_CLASSES entries); with b == NULL
 * the built-in defaults. */
hg_status hg_batch_get_schedule(hg_batch b, hg_schedule* sched);

/* ------------------------------------------------------------ move sequences
 * Exact gains of an ordered sequence of moves (section "Parallel Gain
 * Calculation", subsection "Parallel Gain Recalculation" and its Lemma): the
 * km1 decrease of each move as if the moves were performed one after the
 * other in the given order, computed in parallel from, per (net, block), the
 * largest index of a move out of the block, the smallest index of a move into
 * it and the number of moves out of it.  The best prefix of such a sequence
 * (section "Direct k-way FM": a prefix sum and a reduction).  And the
 * monotone label-propagation round built from both.  Each vertex may appear
 * at most once in a sequence (as in one FM round). */

/* Bytes of the workspace of the calls below for a graph with n vertices and
 * m nets at k blocks: 16 bytes per (net, block) cell (three int32 and a
 * pad), sort and scan buffers.  0 for unsupported arguments.  Any contents
 * are fine on entry. */
size_t hg_moves_workspace_size(int32_t n, int32_t m, int32_t k);

/* gains[j] (int64, device) = km1 before move j minus km1 after it, when the
 * moves 0..j are applied in order to the partition `part` whose pin counts
 * are `phi` (the state BEFORE the sequence; neither is changed).  Move j
 * takes vertex move_u[j] from part[move_u[j]] to block move_to[j].  A vertex
 * twice, a target outside [0,k) or equal to the vertex's block raises the
 * device flag that hg_sync_status reports (such moves contribute nothing). */
hg_status hg_move_gains(hg_graph g, int32_t k, const int32_t* part, const int32_t* phi,
                        int32_t t, const int32_t* move_u, const int32_t* move_to,
                        int64_t* gains, void* workspace, size_t ws_bytes, void* stream);

/* The best prefix of a move sequence: the length p in [0, t] with the largest
 * total gains[0] + ... + gains[p-1] among the prefixes after which every block
 * weight (block_w, the weights before the sequence, plus the moves' vertex
 * weights) is at most max_block_w; the empty prefix always qualifies; ties go
 * to the longer prefix.  best_len[0] (int32) and best_gain[0] (int64) are
 * device outputs.  One workgroup; k <= 256. */
hg_status hg_best_prefix(hg_graph g, int32_t k, int64_t max_block_w, const int32_t* part,
                         const int64_t* block_w, int32_t t, const int32_t* move_u,
                         const int32_t* move_to, const int64_t* gains, int32_t* best_len,
                         int64_t* best_gain, void* workspace, size_t ws_bytes, void* stream);

/* One monotone label-propagation round: candidates and approval as in
 * hg_lp_round, then the approved moves, ordered by (select gain desc, vertex
 * id asc), get their exact gains in that order (hg_move_gains) and only the
 * prefix with the largest total gain is applied (ties: the longer).  Every
 * prefix of approved moves respects L_max, so km1 never increases; the round
 * record's `approved` is the applied prefix and km1_delta its total exact
 * gain.  Arguments as hg_lp_round plus the move workspace. */
hg_status hg_lp_round_exact(hg_graph g, int32_t k, int64_t max_block_w, int32_t* part,
                            int32_t* phi, uint32_t* netstate, int64_t* block_w, uint8_t* eligible,
                            uint8_t* moved, int64_t* km1, hg_round_stats* stats, void* workspace,
                            size_t ws_bytes, void* stream);

/* hg_refine with monotone rounds (direct launches). */
hg_status hg_refine_exact(hg_graph g, int32_t k, double eps, int32_t rounds, int32_t* part,
                          int32_t* phi, uint32_t* netstate, int64_t* block_w, uint8_t* eligible,
                          hg_round_stats* stats, int64_t* km1_out, void* workspace,
                          size_t ws_bytes, void* stream);

/* -------------------------------------------------------------- rebalancing
 * Section "Rebalancing": move vertices out of blocks heavier than L_max,
 * non-negative gains first, then the smallest losses.  Deterministic
 * synchronous rounds; each round, from the round-start state:
 *   1. every vertex u of an overloaded block a (c(V_a) > L_max) picks the
 *      best block i != a with c(V_i) + c(u) <= L_max -- any block, not only
 *      neighbouring ones -- by (g_i(u) desc, c(V_i) asc, i asc); gains may
 *      be negative; no such block: no candidate;
 *   2. per source block a, the candidates in (gain desc, id asc) order: the
 *      shortest prefix whose weight reaches the excess c(V_a) - L_max is
 *      proposed (all of them if their total falls short);
 *   3. per target block t, the proposals in (gain desc, id asc) order: the
 *      longest prefix with c(V_t) + prefix weight <= L_max is applied;
 *   4. pins of nets holding a moved vertex become eligible (others keep
 *      their flag); moved[u] = 1 for the moved vertices, 0 for the rest.
 * No block within L_max leaves it and no overloaded block gets heavier; a
 * balanced partition is left as it is.  The round record (hg_round_stats)
 * reads: eligible = vertices considered (in overloaded blocks), boundary =
 * moves proposed, candidates = vertices with a target, approved = moves
 * applied, active_pins = sum of d(u) over the considered vertices; the other
 * fields as for a label-propagation round (km1_delta is negative when km1
 * grows).
 * ------------------------------------------------------------------------ */

/* Bytes of the rebalancing workspace (device, 256-byte aligned) for n
 * vertices and k blocks (it holds a gain cache); 0 on bad arguments. */
size_t hg_rebalance_workspace_size(int32_t n, int32_t k);

/* `rounds` rebalancing rounds on the caller's state (the buffers of
 * hg_lp_round, describing part: hg_compute_pincounts or earlier rounds
 * establish that), against L_max = max_block_w; stats gets one record per
 * round (rounds after balance is restored, or after a round that moved
 * nothing, are empty).  moved is required. */
hg_status hg_rebalance(hg_graph g, int32_t k, int64_t max_block_w, int32_t rounds, int32_t* part,
                       int32_t* phi, uint32_t* netstate, int64_t* block_w, uint8_t* eligible,
                       uint8_t* moved, int64_t* km1, hg_round_stats* stats, void* workspace,
                       size_t ws_bytes, void* stream);

/* -------------------------------------------------------------- contraction
 * Section "Coarsening", subsection "Contraction": contract a clustering of
 * the vertices of a loaded hypergraph into a coarse hypergraph.
 *   cluster  int32[n]   cluster id of every vertex, in [0, n) (ids need not
 *                       be consecutive; an id out of range raises the error
 *                       flag that hg_sync_status reports)
 * Outputs (device, caller-owned, capacities from the fine sizes):
 *   map      int32[n]     coarse vertex of every vertex: the rank of its
 *                         cluster id among the used ids (increasing order)
 *   cvwgt    int32[n]     c'(x) = sum of c(v) over map[v] = x (first n'
 *                         entries; a sum >= 2^31 raises the error flag)
 *   ceptr    int64[m+1]   coarse net CSR offsets (first m' + 1 entries)
 *   cpins    int32[P]     coarse pins, increasing within each net (first P')
 *   cewgt    int32[m]     coarse net weights (first m')
 *   sizes    int64[3]     n', m', P'
 * A coarse net is a fine net with its pins mapped and duplicates removed;
 * nets left with one pin are dropped; nets with the same pin set become one
 * net whose weight is the sum, placed at the lowest fine net id among them;
 * coarse nets are numbered in increasing order of that id.  m' may be 0.
 * Identical nets are found with the paper's fingerprints (sum of v^2, with
 * the size) and pin-by-pin comparison.  km1 of any partition of the coarse
 * hypergraph equals km1 of its projection through map.  hg_load_csr on the
 * outputs (when m' >= 1) gives the coarse graph handle (incidence arrays).
 * Requires P < 2^31.  The workspace (device, 256-byte aligned) is
 * hg_contract_workspace_size(n, m, P) bytes.
 * ------------------------------------------------------------------------ */
size_t hg_contract_workspace_size(int32_t n, int32_t m, int64_t P);

hg_status hg_contract(hg_graph g, const int32_t* cluster, int32_t* map, int32_t* cvwgt,
                      int64_t* ceptr, int32_t* cpins, int32_t* cewgt, int64_t* sizes,
                      void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ serving
 * A request server.  Refinement jobs arrive over time.  Each is admitted
 * into a caller-provided device arena once its exact footprint
 * (hg_request_bytes) fits, in arrival order.  Admitted jobs are loaded (copied
 * in, checked, incidence built) on their own stream and host thread, then
 * advanced together one label-propagation round per step in batched launches:
 * continuous batching, where a job joins at the next step after its load and
 * leaves after its last round, and its partition state stays in device memory
 * in between.  Every result is bit-identical to hg_refine on the job alone.
 * The server keeps two host threads (loader and executor) and two streams of
 * default priority; it allocates no device memory. */

typedef struct hg_server_s* hg_server;

/* One refinement job.  Every array is HOST memory and must stay valid until
 * the job is done; page-locked memory (hipHostMalloc) lets the copies run
 * asynchronously, pageable memory makes them block the server's threads. */
typedef struct {
  int32_t n, m;
  int64_t P;
  const int64_t* eptr;        /* [m+1] net CSR offsets                          */
  const int32_t* pins;        /* [P]                                            */
  const int32_t* vwgt;        /* [n] or NULL (unit)                             */
  const int32_t* ewgt;        /* [m] or NULL (unit)                             */
  const int32_t* part;        /* [n] start partition, ids in [0,k)              */
  int32_t k;                  /* 2..256                                         */
  int32_t rounds;             /* label-propagation rounds, 1..1024              */
  double eps;                 /* 0 < eps < 1                                    */
  int32_t* part_out;          /* OUT [n] final partition, or NULL               */
  hg_round_stats* stats_out;  /* OUT [rounds] round records, or NULL            */
  int64_t* km1_out;           /* OUT [1] final km1, or NULL                     */
  double arrival_ms;          /* scheduled arrival on the server clock (latency
                                 is measured from it, not from the submit)      */
} hg_request;

#define HG_REQ_PENDING 0      /* waiting for memory or a slot                   */
#define HG_REQ_ADMITTED 1     /* memory reserved, being loaded                  */
#define HG_REQ_ACTIVE 2       /* loaded, in the batch                           */
#define HG_REQ_DONE 3         /* finished (status says how)                     */

typedef struct {
  int32_t state;              /* HG_REQ_*                                       */
  int32_t status;             /* HG_OK, or the error that ended the job         */
  double arrival_ms;          /* server clock, milliseconds since creation      */
  double admit_ms;            /* memory reserved                                */
  double loaded_ms;           /* loaded and checked                             */
  double done_ms;             /* its last result copy finished on the GPU       */
  int64_t footprint;          /* device bytes held while admitted               */
  int64_t first_step;         /* server step of its first round                 */
} hg_request_info;

typedef struct {
  int64_t submitted, completed, failed;
  int64_t steps;              /* batched rounds launched                        */
  int64_t member_rounds;      /* sum over steps of the members in the step      */
  int64_t pin_rounds;         /* sum over steps of the members' pin counts      */
  int64_t max_members;        /* most members in one step                       */
  int64_t rebuilds;           /* work-table rebuilds (membership changes)       */
  int64_t peak_bytes;         /* most arena bytes held by admitted jobs         */
} hg_server_stats;

/* Device bytes a job of this shape holds while admitted: its net CSR,
 * incidence CSR, workspace (hg_workspace_size with k_max = k), partition
 * state (part, Phi, net state, block weights, km1, eligible flags) and round
 * records, each 256-byte aligned.  0 for unsupported sizes. */
size_t hg_request_bytes(int32_t n, int32_t m, int64_t P, int32_t k, int32_t rounds,
                        int32_t weighted_vertices, int32_t weighted_nets);

/* Start a server on device memory [arena, arena + arena_bytes): the first
 * table_bytes hold the batched work tables, the rest is the jobs' memory.  At
 * most max_active jobs are admitted at once.  big_pins > 0 opens a second
 * lane (own stream and tables) for jobs of at least big_pins pins, so that
 * smaller jobs never wait for their rounds; 0 keeps one lane.  Each lane takes
 * half of the table region, split into two halves rebuilt alternately.
 * sched: HG_SIZE_CLASSES schedules or NULL: then one unit per work item in
 * every class (a server step usually holds a few jobs, so the most
 * workgroups per job).  The current device at the call is the server's
 * device. */
hg_status hg_server_create(void* arena, size_t arena_bytes, size_t table_bytes,
                           int32_t max_active, int64_t big_pins, const hg_schedule* sched,
                           hg_server* out);

/* Queue a job (copied; its arrays are read later).  Checks the arguments on
 * the host; a job whose footprint exceeds the job memory ends with
 * HG_ERR_WORKSPACE, one whose arrays fail the load checks with
 * HG_ERR_INVALID or HG_ERR_UNSUPPORTED (see hg_server_info).  *id numbers
 * the jobs 0, 1, 2, ... in submission order.  Thread-safe. */
hg_status hg_server_submit(hg_server s, const hg_request* r, int64_t* id);

/* Milliseconds since hg_server_create on the server clock. */
double hg_server_now_ms(hg_server s);

/* State and timestamps of job `id`. */
hg_status hg_server_info(hg_server s, int64_t id, hg_request_info* out);

/* Wait until every submitted job is done or timeout_ms passed (< 0: no
 * limit); *outstanding (may be NULL) receives the number not yet done. */
hg_status hg_server_drain(hg_server s, double timeout_ms, int64_t* outstanding);

hg_status hg_server_get_stats(hg_server s, hg_server_stats* out);

/* Finish every submitted job, stop the threads, release host resources. */
void hg_server_free(hg_server s);

#ifdef __cplusplus
}
#endif
#endif /* HGREF_H */
