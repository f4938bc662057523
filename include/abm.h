/*
 * abm.h -- C ABI of libabm.so, an MI355X (gfx950) implementation of the ABMax
 * hot path (arXiv 2508.16508): distinct updates to a dynamically selected,
 * variable-size subset of agents held in fixed-capacity struct-of-arrays
 * slots, and the wolf-sheep-grass predation step built on it.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers are DEVICE pointers unless marked (host).  Structs passed by
 *    pointer (abm_soa, abm_records, parameter blocks) live in host memory and
 *    are read during the call only.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every call is asynchronous on that stream and never synchronises the
 *    device; counts are written to device scalars so a caller reads them when
 *    it chooses.  Calls sharing a workspace must be ordered on one stream.
 *  - The caller owns every buffer.  The library keeps no pointer after a call
 *    returns and allocates nothing in these calls.
 *  - Status codes: ABM_OK, or a negative code with a message available from
 *    abm_last_error() (thread-local).  Argument errors are detected on the host
 *    before anything is launched, so a failed call has no effect.
 *  - Masks are uint8 arrays: a non-zero byte selects.  `alive` arrays are
 *    int32: non-zero = live slot, 0 = free placeholder slot (Sec. 4: shapes stay
 *    fixed, unused capacity is held by placeholder agents).
 *  - Sizes: capacities, counts and grids must be below 2^31.
 */
#ifndef ABM_H
#define ABM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ABM_MAX_ATTRS 16

#if defined(__GNUC__)
#define ABM_API __attribute__((visibility("default")))
#else
#define ABM_API
#endif

enum {
    ABM_OK = 0,
    ABM_E_INVALID = -1,     /* bad argument (NULL pointer, size out of range, mismatch) */
    ABM_E_WORKSPACE = -2,   /* workspace missing or smaller than abm_workspace_bytes() */
    ABM_E_HIP = -3,         /* a HIP runtime call or kernel launch failed */
    ABM_E_UNSUPPORTED = -4  /* current device is not gfx950 */
};

/* A collection of agents (the paper's Set, Sec. 2): n_attrs int32 attribute
 * arrays, each of `capacity` elements (struct of arrays), plus an optional
 * `alive` array of `capacity` int32.  Attribute arrays must not alias each
 * other, the alive array, or any record/mask argument of the same call. */
typedef struct abm_soa {
    int32_t n_attrs;                 /* 1..ABM_MAX_ATTRS */
    int64_t capacity;                /* number of slots, 0 <= capacity < 2^31 */
    int32_t* attr[ABM_MAX_ATTRS];    /* device, attr[a][slot] */
    int32_t* alive;                  /* device, may be NULL where not used */
} abm_soa;

/* Dense update records, struct of arrays: record j is (attr[0][j], ...). */
typedef struct abm_records {
    int32_t n_attrs;                 /* must equal the destination's n_attrs */
    int64_t count;                   /* m, 0 <= m < 2^31 */
    const int32_t* attr[ABM_MAX_ATTRS];
} abm_records;

/* Operations, for abm_workspace_bytes(). */
enum {
    ABM_OP_SELECT_UPDATE = 1,
    ABM_OP_ADD_AGENTS = 2,
    ABM_OP_REMOVE_AGENTS = 3,
    ABM_OP_SELECT_INDICES = 4,
    ABM_OP_PREDATION = 5
};

/* Bytes of workspace `op` needs for `capacity` slots (for ABM_OP_SELECT_UPDATE
 * with an update mask, pass capacity = max(slots, records)).  For
 * ABM_OP_PREDATION pass capacity = max(cap_s, cap_w).  A larger workspace is
 * always accepted; one workspace sized for the largest use serves every op. */
ABM_API size_t abm_workspace_bytes(int op, int64_t capacity);

/* Zero-fill a workspace before its first use (it holds the single-pass scan's
 * tile ticket and tile status words, which later calls keep consistent).  Must
 * be called once per workspace allocation, outside any graph capture. */
ABM_API int abm_workspace_init(void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * abm_select_update -- distinct updates to a dynamically selected subset.
 * Sec. 4 (the toy task and the Rank-Match / Sort-Count-Iterate algorithms):
 * p = number of selected slots, q = number of selected records, r = min(p, q);
 * the j-th selected slot in ascending order receives every attribute of the
 * j-th selected record in ascending order, for j < r.  Nothing else changes.
 *
 *   dst        destination collection (alive not used).
 *   sel_mask   device uint8[dst->capacity], non-zero = slot selected.
 *   upd        records; upd->n_attrs == dst->n_attrs.
 *   upd_mask   NULL: all upd->count records are selected (q = count).
 *              else device uint8[upd->count], non-zero = record selected.
 *   d_applied  device int64: r.
 *   d_dropped  device int64 or NULL: q - r (records that found no slot).
 *   ws         workspace of at least abm_workspace_bytes(ABM_OP_SELECT_UPDATE,
 *              max(capacity, upd->count)) bytes, initialised once.
 * Applying the same call twice gives the same state as applying it once.
 * ------------------------------------------------------------------------- */
ABM_API int abm_select_update(const abm_soa* dst, const uint8_t* sel_mask, const abm_records* upd,
                      const uint8_t* upd_mask, int64_t* d_applied, int64_t* d_dropped,
                      void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * abm_select_update_noalloc -- abm_select_update (dense records: every record
 * is selected, as with upd_mask == NULL) for callers that cannot allocate:
 * code under stream capture, tight serving loops, harnesses that forbid
 * device allocation.  It takes no workspace and allocates nothing; its scan
 * state lives in a static device array of the library (under 512 KiB per
 * device, held until the process ends).  Same semantics, arguments and
 * results as abm_select_update, plus:
 *   dst->capacity  at most 2^28 slots, else ABM_E_INVALID before any launch.
 *   d_error        device int64 or NULL: receives 1 if a bounded wait of the
 *                  scan gave up since the last call that passed d_error (the
 *                  results are then invalid; never expected), else 0.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (different streams, or host threads) race and give wrong
 * results; serialise them.
 * ------------------------------------------------------------------------- */
ABM_API int abm_select_update_noalloc(const abm_soa* dst, const uint8_t* sel_mask,
                                      const abm_records* upd, int64_t* d_applied,
                                      int64_t* d_dropped, int64_t* d_error, void* stream);

/* ---------------------------------------------------------------------------
 * abm_select_indices -- the paper's select_agents (Sec. 2): the ascending
 * indices of the selected slots and their number.
 *   mask       device uint8[n].
 *   out_idx    device int32[n]; entries [0, k) are written, the rest untouched.
 *   d_count    device int64: k.
 * ------------------------------------------------------------------------- */
ABM_API int abm_select_indices(const uint8_t* mask, int64_t n, int32_t* out_idx, int64_t* d_count,
                       void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * abm_add_agents -- new agents with distinct initial states (Sec. 1 and the
 * Sec. 4 toy task applied to free slots): free slots are those with
 * alive == 0; newborn j (record j) goes to the j-th lowest free slot, for
 * j < min(#free, count), and that slot's alive becomes 1.
 *   dst        collection; dst->alive required.
 *   newborn    records, n_attrs == dst->n_attrs.
 *   d_added    device int64: number placed.
 *   d_dropped  device int64 or NULL: newborns that found no free slot.
 * ------------------------------------------------------------------------- */
ABM_API int abm_add_agents(const abm_soa* dst, const abm_records* newborn, int64_t* d_added,
                   int64_t* d_dropped, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * abm_remove_agents -- the paper's set_agents_mask (Sec. 2): an independent,
 * non-conflicting masked update.  alive[i] = 0 wherever kill_mask[i] != 0;
 * other attributes of a removed slot are left as they were.
 *   kill_mask  device uint8[dst->capacity].
 *   d_removed  device int64: number of slots that were live and are now free.
 * ------------------------------------------------------------------------- */
ABM_API int abm_remove_agents(const abm_soa* dst, const uint8_t* kill_mask, int64_t* d_removed,
                      void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * abm_resolve_conflicts -- many claimants for one resource (Sec. 1; Sec. 5.2
 * resolves competing moves with a priority per claimant).  Claim c is active
 * when active == NULL or active[c] != 0, and its target lies in
 * [0, n_targets); other claims are ignored.  With key_c = prio_c * 2^32 + c:
 *   best[t]   = minimum key over active claims on t, or UINT64_MAX if none
 *   winner[t] = claim index of best[t], or -1
 *   won[c]    = 1 for the claim holding best[target_c], else 0.
 * The lowest priority wins; equal priorities go to the lower claim index.
 *   target    device int32[n_claims]; prio device uint32[n_claims];
 *   active    device uint8[n_claims] or NULL;
 *   best      device uint64[n_targets] (overwritten; no reset needed);
 *   winner    device int32[n_targets]; won device uint8[n_claims].
 * 0 <= n_claims < 2^31 (claim indices fit winner[]'s int32), else
 * ABM_E_INVALID before any launch.  No workspace.
 * ------------------------------------------------------------------------- */
ABM_API int abm_resolve_conflicts(int64_t n_claims, const int32_t* target, const uint32_t* prio,
                          const uint8_t* active, int64_t n_targets, uint64_t* best,
                          int32_t* winner, uint8_t* won, void* stream);

/* ---------------------------------------------------------------------------
 * Predation model (Sec. 5.1, Fig. 2: Wilensky's wolf-sheep-grass on a 2-D
 * toroidal lattice).  Each step runs, in order:
 *   move   every live agent steps to a uniformly drawn one of its 8 neighbours
 *          and pays 1 energy;
 *   eat    grass: on each grown cell holding live sheep, the sheep with the
 *          lowest key (draw << 32 | slot) eats (+gain_s, countdown = R);
 *          prey: on each cell holding live sheep and live wolves, the
 *          lowest-key sheep is eaten by the lowest-key wolf (+gain_w); with
 *          multi_prey = 1, for every r below min(#sheep, #wolves) of the
 *          cell the r-th sheep in key order is eaten by the r-th wolf in key
 *          order (the rank-and-match of Sec. 4, Alg. 1, per cell);
 *   breed  live agents with energy > 0 and draw < T reproduce: the j-th
 *          breeder (ascending slot) puts a child on its own cell into the
 *          j-th lowest free slot; child energy e >> 1, parent keeps the rest;
 *   die    live agents with energy < 0 become free slots;
 *   regrow every countdown above zero drops by one.
 * Draws are hi32(mix64(mix64(seed << 32 | step) ^ (agent << 32 | purpose)))
 * with mix64 the SplitMix64 output function, so a model resumes exactly from
 * its state and step counter.
 * ------------------------------------------------------------------------- */
typedef struct abm_predation_params {
    int32_t W, H;          /* lattice, cell = y * W + x; 1 <= W, H; W * H < 2^31 */
    int32_t R;             /* regrowth delay in steps, >= 1 */
    int32_t gain_s, gain_w;
    uint32_t T_s, T_w;     /* reproduce when draw < T (floor(prob * 2^32)) */
    uint32_t seed;
    int64_t cap_s, cap_w;  /* slot capacities, 1 <= cap < 2^31 */
    int64_t n_s0, n_w0;    /* initial live agents (slots 0 .. n0-1), n0 <= cap */
    int32_t multi_prey;    /* 0: one prey per cell; 1: prey matched by rank within a cell */
} abm_predation_params;

typedef struct abm_species {
    int32_t* x;            /* device int32[cap] */
    int32_t* y;
    int32_t* e;            /* energy */
    int32_t* alive;
} abm_species;

typedef struct abm_predation_state {
    int32_t* grass;        /* device int32[W*H]: steps until regrown (0 = grown) */
    abm_species sheep, wolves;
    uint64_t* claims;      /* device uint64[3 * W*H], scratch owned by the caller */
    int64_t* stats;        /* device int64[8 * n_steps] or NULL: per step
                              live_s, live_w (at step start), grass_eaten,
                              sheep_eaten, births_s, births_w, starved_s, starved_w */
    uint32_t step;         /* (host) index of the next step; advanced by the call */
} abm_predation_state;

/* Fill the initial state: each cell grown with probability 1/2, else a
 * countdown uniform in [1, R]; agents in slots 0 .. n0-1 at uniform cells with
 * energy uniform in [0, 2 * gain); all other slots zero.  Sets s->step = 0. */
ABM_API int abm_predation_init(const abm_predation_params* p, abm_predation_state* s, void* stream);

/* Run n_steps steps starting at s->step, then advance s->step.  When
 * s->stats is non-NULL, row k of it receives the statistics of step k of this
 * call.  ws: abm_workspace_bytes(ABM_OP_PREDATION, max(cap_s, cap_w)). */
ABM_API int abm_predation_step(const abm_predation_params* p, abm_predation_state* s, int32_t n_steps,
                       void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Batched primitives: many independent collections of uneven sizes, packed
 * back to back, each processed exactly as the single-collection call above
 * would process it alone (the paper vectorises its manipulation functions
 * over Sets, Sec. 2).  Segment m owns slots [slot_off[m], slot_off[m+1]) of
 * the packed collection and records [rec_off[m], rec_off[m+1]) of the packed
 * records.  Offsets are DEVICE int64 arrays of n_segments + 1 entries,
 * non-decreasing, with slot_off[0] = 0, slot_off[n_segments] = capacity and
 * rec_off[n_segments] <= record count (results are undefined otherwise).
 * Counts are device int64 arrays of n_segments entries.  Workspace: as for
 * the single call with capacity = the packed slot count.
 * ------------------------------------------------------------------------- */
ABM_API int abm_select_update_batched(int32_t n_segments, const abm_soa* dst,
                                      const int64_t* slot_off, const uint8_t* sel_mask,
                                      const abm_records* upd, const int64_t* rec_off,
                                      int64_t* d_applied, int64_t* d_dropped, void* ws,
                                      size_t ws_bytes, void* stream);

ABM_API int abm_add_agents_batched(int32_t n_segments, const abm_soa* dst, const int64_t* slot_off,
                                   const abm_records* newborn, const int64_t* rec_off,
                                   int64_t* d_added, int64_t* d_dropped, void* ws,
                                   size_t ws_bytes, void* stream);

ABM_API int abm_remove_agents_batched(int32_t n_segments, const abm_soa* dst,
                                      const int64_t* slot_off, const uint8_t* kill_mask,
                                      int64_t* d_removed, void* ws, size_t ws_bytes,
                                      void* stream);

/* Claims [claim_off[m], claim_off[m+1]) compete for targets
 * [target_off[m], target_off[m+1]) of the packed best/winner arrays; target[c]
 * is segment-local, the key uses the segment-local claim index, and winner[t]
 * holds that local index (or -1). */
ABM_API int abm_resolve_conflicts_batched(int32_t n_segments, const int64_t* claim_off,
                                          int64_t n_claims, const int32_t* target,
                                          const uint32_t* prio, const uint8_t* active,
                                          const int64_t* target_off, int64_t n_targets,
                                          uint64_t* best, int32_t* winner, uint8_t* won,
                                          void* stream);

/* ---------------------------------------------------------------------------
 * Batched predation: many independent models of uneven sizes advanced by one
 * persistent launch (the paper vectorises identical models, Sec. 2 and
 * Table 2; here shapes may differ).  Every model follows exactly the one-model
 * definition above with its own parameters and seed, so each model's state
 * is bit-identical to running it alone.
 *
 * Packed layout: model m owns cells [cell_off, cell_off + W*H) of `ready`
 * (one int32 per cell) and of `claims` (three uint64 per cell), and slots
 * [sheep_off, sheep_off + cap_s) / [wolf_off, wolf_off + cap_w) of the species
 * arrays.  Ranges must not overlap.  `ready` holds the step at which a cell is
 * grown again (grown at step t iff ready <= t); abm_predation_batched_grass
 * converts it to the countdown form of abm_predation_state.  A model with
 * multi_prey set links its agents into per-cell lists through slots
 * [sheep_off, sheep_off + cap_s) of link_s and [wolf_off, wolf_off + cap_w)
 * of link_w; a run leaves such a model untouched and sets the workspace error
 * word if the batch has no links.
 * ------------------------------------------------------------------------- */
typedef struct abm_model_desc {   /* device array; the library updates the last five fields */
    int32_t W, H, R, gain_s, gain_w;
    uint32_t T_s, T_w, seed;
    int32_t multi_prey;            /* 0: one prey per cell; nonzero: prey matched by rank within a
                                      cell (as abm_predation_params; needs the batch's links) */
    int64_t cap_s, cap_w;          /* each in [1, 2^30] */
    int64_t n_s0, n_w0;
    int64_t cell_off, sheep_off, wolf_off;
    int32_t step;                  /* steps done so far (0 after init) */
    int32_t steps_target;          /* a run stops advancing the model here */
    int64_t updates;               /* sum over steps run of live agents at step start */
    int64_t live_s, live_w;        /* live agents after the last run */
} abm_model_desc;

typedef struct abm_batch {        /* host struct of device pointers */
    int32_t n_models;              /* 0 .. 65535 */
    int64_t max_cap;               /* max over models of max(cap_s, cap_w) */
    abm_model_desc* models;        /* device abm_model_desc[n_models] */
    int32_t* ready;                /* device int32[sum of W*H] */
    uint64_t* claims;              /* device uint64[3 * sum of W*H]; set by init, kept all-ones between runs */
    abm_species sheep, wolves;     /* device int32[sum of caps] each */
    int32_t* link_s;               /* device int32[sum of cap_s] and [sum of cap_w]: per-cell lists */
    int32_t* link_w;               /* of multi-prey models (scratch; NULL if no model has multi_prey) */
} abm_batch;

typedef struct abm_tuning {
    int32_t block_threads;         /* threads per model workgroup (multiple of 64 in [256, 1024]); 0 = 512 */
    int32_t workgroups;            /* persistent workgroups; 0 = as many as are resident at once */
    int32_t items;                 /* slots per thread per chunk: 1, 2 or 4; 0 = 4 */
    int32_t team_size;             /* workgroups per team (1..16); 0 or 1 = no teams */
    int32_t team_models;           /* the first team_models entries of order run in teams */
    int32_t team_workgroups;       /* workgroups formed into teams, a multiple of 8 * team_size;
                                      0 = enough for team_models teams (capped by residency) */
    int32_t global_claims;         /* nonzero: every claim table in global memory; 0 = models
                                      of one workgroup whose table fits keep it in LDS
                                      (abm_batched_lds_cells) */
} abm_tuning;

/* Workspace for abm_predation_run_batched with at most n_workgroups
 * workgroups: a 256-byte header, a fixed team area and a breeder list per
 * workgroup.  The header ends with an error word (offset 248) that a run sets
 * to 1 if some descriptor's cap_s + cap_w exceeds 2 * max_cap (that model is
 * then left untouched) or if a team barrier times out (a member never ran;
 * the state of that team's model is then undefined).  The error word is
 * sticky: zero the workspace once with abm_workspace_init before its first
 * run; runs only ever set the word.  Returns 0 for max_cap outside
 * [1, 2^30] or n_workgroups outside [1, 8192]. */
ABM_API size_t abm_batched_workspace_bytes(int64_t max_cap, int32_t n_workgroups);

/* Initial state of every model (the one-model definition per model, with the
 * model's seed); descriptors must hold step = 0 and updates = 0. */
ABM_API int abm_predation_batched_init(const abm_batch* b, void* stream);

/* Advance every model by min(max_steps, steps_target - step) steps.  order is
 * a device int32 permutation of [0, n_models): workgroups take models in that
 * order (largest first balances the load).  With tune->team_size K > 1 the
 * first tune->team_models entries of order are each advanced by a team of K
 * workgroups that split the model's slots into K contiguous ranges and meet
 * at three device-wide team barriers per step; the results are the same as
 * with one workgroup per model.  Teams need 8 K resident workgroups (else
 * ABM_E_INVALID).  Claim tables of small models are kept in LDS unless
 * tune->global_claims is set (abm_batched_lds_cells).  The workspace must hold abm_batched_workspace_bytes(max_cap,
 * n) bytes, n being the number of workgroups launched: at most the resident
 * count (or tune->workgroups), which the caller can use as the bound.
 * Afterwards each descriptor's step, updates, live_s and live_w are current. */
ABM_API int abm_predation_run_batched(const abm_batch* b, const int32_t* order, int32_t max_steps,
                                      const abm_tuning* tune, void* ws, size_t ws_bytes,
                                      void* stream);

/* Largest W * H whose claim table (three uint64 per cell, 24 bytes) fits in
 * the LDS that abm_predation_run_batched gives each workgroup at this launch
 * shape on the current device: the CU's LDS shared among the workgroups
 * resident at block_threads threads, less the kernel's own, so that no
 * workgroup is displaced for it.  0 if no supported device is current or the
 * shape is invalid.  Models advanced by one workgroup (not a team) whose table
 * fits post, read and clear their claims in LDS; the results are the same as
 * with the global table, whose cells of these models are left untouched
 * (all-ones). */
ABM_API int64_t abm_batched_lds_cells(int32_t block_threads, int32_t items);

/* countdown[cell_off + c] = max(0, ready[cell_off + c] - step) for every model:
 * the grass array of the one-model state.  countdown: device int32[sum of W*H]. */
ABM_API int abm_predation_batched_grass(const abm_batch* b, int32_t* countdown, void* stream);

/* ---------------------------------------------------------------------------
 * Captured rollouts (Sec. 2: the paper compiles multi-step rollouts of
 * vectorised models once and runs them as one scan; here a rollout is
 * captured once as a HIP graph and replayed with one launch).
 *
 * abm_predation_batched_graph records n_chunks consecutive launches of
 * abm_predation_run_batched(b, order, chunk_steps, tune, ws, ws_bytes) --
 * each advances every model by up to chunk_steps steps, never past its
 * steps_target -- into a graph, on a capture stream of its own, and returns
 * an executable handle in *out.  Nothing runs at capture.  Argument errors
 * are those of abm_predation_run_batched (checked at capture; no handle is
 * returned).  The handle owns the graph only: every device pointer reachable
 * from b, order and ws is recorded as it is, so those buffers must stay
 * allocated and unmoved until abm_graph_destroy; their contents may change
 * between replays (a replay continues from the current state and step
 * counters).  abm_graph_replay launches the graph on `stream` (asynchronous,
 * stream-ordered; the device must be the one current at capture).
 * abm_graph_destroy releases the handle (NULL is accepted).
 * ------------------------------------------------------------------------- */
typedef struct abm_graph_s abm_graph;

ABM_API int abm_predation_batched_graph(const abm_batch* b, const int32_t* order, int32_t chunk_steps,
                                        int32_t n_chunks, const abm_tuning* tune, void* ws,
                                        size_t ws_bytes, abm_graph** out);
ABM_API int abm_graph_replay(abm_graph* g, void* stream);
ABM_API int abm_graph_destroy(abm_graph* g);

/* ---------------------------------------------------------------------------
 * sort_agents and select_agents (Sec. 2 API list).
 * ------------------------------------------------------------------------- */

/* Workspace bytes for abm_sort_agents over n agents permuting n_cols columns
 * (the attributes, plus alive when it is non-NULL), or for abm_select_agents
 * with n_cols = 0: 4 n for the permutation, max(12 n, n x record) where a
 * record is n_cols int32 rounded up to a power of two, and the tile counts
 * (about n / 4).  0 for n outside [0, 2^31) or n_cols outside [0, 17]. */
ABM_API size_t abm_sort_workspace_bytes(int64_t n, int32_t n_cols);

/* Reorder the collection by a runtime key (Sec. 2 sort_agents): afterwards
 * position j holds the agent that had the j-th smallest key (descending != 0:
 * the j-th largest); agents with equal keys keep their index order.  Every
 * attribute column and, if non-NULL, alive are permuted in place.  key: device
 * int32[capacity].  perm (device int32[capacity], may be NULL) receives the old
 * index of the agent now at each position.  ws: device, 256-byte aligned, at
 * least abm_sort_workspace_bytes(capacity, n_attrs + (alive != NULL)) bytes
 * (else ABM_E_WORKSPACE); its contents on entry do not matter. */
ABM_API int abm_sort_agents(const abm_soa* dst, const int32_t* key, int32_t descending,
                            int32_t* perm, void* ws, size_t ws_bytes, void* stream);

/* Sec. 2 select_agents: order (device int32[n]) receives the indices i with
 * cond[i] != 0 in increasing order, then the others in increasing order;
 * *d_count (device int64) the number of the former.  ws: device, 256-byte
 * aligned, at least abm_sort_workspace_bytes(n, 0) bytes. */
ABM_API int abm_select_agents(const uint8_t* cond, int64_t n, int32_t* order, int64_t* d_count,
                              void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Limit order books with batch matching (Sec. 5.3, Fig. 5), many books at
 * once (the paper vectorises the matching over books, Table 4).  A book holds
 * up to cap orders (side 0 buy / 1 sell, price in ticks, qty, time = step
 * placed, alive) and a last price.  Step t of book b, with draws keyed on
 * (seed + b, t, trader, purpose):
 *   expiry   orders placed expiry or more steps ago are cancelled;
 *   orders   trader k < traders orders when its draw < T_order: a buy or a
 *            sell with probability 1/2 each, at last + u - spread (u uniform
 *            on [0, 2 spread], clamped to [1, 2^24 - 1]), for 1 + (uniform
 *            on [0, max_qty)) shares; the new orders, in trader order, take
 *            the lowest free slots; those finding none are dropped;
 *   matching buys in price-time priority (price descending, then time, then
 *            slot), sells with price ascending; CB, CS the cumulative shares
 *            along those lists; matched volume V = max over buys r of
 *            min(CB_r, CS(p_r)), CS(p) = shares of the sells priced at most
 *            p; every order fills the part of its share range below V
 *            (filled orders are removed, partly filled ones keep the rest);
 *            the last price becomes the floor of the mean of the buy and sell
 *            prices covering share V (unchanged when V = 0).
 * ------------------------------------------------------------------------- */
typedef struct abm_lob_params {
    int32_t cap;           /* order slots per book, in [1, 1024] */
    int32_t traders;       /* in [0, 1024] */
    uint32_t T_order;      /* a trader orders when its draw < T_order */
    int32_t spread;        /* price offsets on [-spread, spread] ticks, spread in [0, 2^22] */
    int32_t max_qty;       /* quantities on [1, max_qty], max_qty in [1, 2^20] */
    int32_t expiry;        /* an order lives expiry steps, >= 1 */
    int32_t price0;        /* initial last price, in [1, 2^24) */
    uint32_t seed;         /* book b draws with seed + b (mod 2^32) */
} abm_lob_params;

typedef struct abm_lob_state {
    int32_t n_books;       /* in [1, 2^20] */
    int32_t *side, *price, *qty, *time, *alive;   /* device int32[n_books * cap] */
    int32_t* last_price;   /* device int32[n_books] */
    int64_t* stats;        /* device int64[n_steps][n_books][8] or NULL: per step and book
                              buys, sells (live after matching), placed, dropped, expired,
                              volume, filled_orders (fully or partly), price */
    uint32_t step;         /* (host) index of the next step; steps stay below 2^24 */
} abm_lob_state;

/* Empty books at price0; sets s->step = 0. */
ABM_API int abm_lob_init(const abm_lob_params* p, abm_lob_state* s, void* stream);

/* Run n_steps steps of every book from s->step, then advance s->step.  One
 * workgroup per book keeps the book in LDS for the whole call. */
ABM_API int abm_lob_step(const abm_lob_params* p, abm_lob_state* s, int32_t n_steps,
                         void* stream);

/* ---------------------------------------------------------------------------
 * Traffic cellular automaton (Sec. 5.2, Fig. 4), many roads at once (the
 * paper vectorises it over roads with different car counts, Table 3).  A road
 * is 3 lanes x length cells; cell (lane, x), x = 0 the entry column, x =
 * length - 1 the exit column.  Cars occupy 3 * length slots (lane, pos,
 * alive).  Step t of road r, with draws keyed on (seed + r, t, agent,
 * purpose):
 *   lights  exit lane l is green iff its draw < T_green;
 *   decide  on the occupancy at the start of the step, a car in the exit
 *           column leaves under green and waits under red; any other car
 *           picks left / straight / right uniformly (off the road means
 *           straight) and claims the cell one column ahead in that lane
 *           unless it is occupied (then it waits);
 *   resolve each claimed cell admits one car, by its priority mask over the
 *           arrival directions: straight, then from the lane below, then
 *           from the lane above; winners move, the others wait;
 *   leave   leaving cars get alive = 0 (their other fields are kept);
 *   spawn   every entry cell free after the moves whose draw < T_spawn gets a
 *           car; the spawned cars, in lane order, take the lowest free slots.
 * ------------------------------------------------------------------------- */
typedef struct abm_traffic_params {
    int32_t length;        /* cells per lane, in [2, 1024] */
    uint32_t T_green;      /* a light is green when its draw < T_green */
    uint32_t T_spawn;      /* a free entry cell spawns a car when its draw < T_spawn */
    uint32_t seed;         /* road r draws with seed + r (mod 2^32) */
} abm_traffic_params;

typedef struct abm_traffic_state {
    int32_t n_roads;       /* in [1, 2^20] */
    int32_t* lane;         /* device int32[n_roads * 3 * length]; road r at [r*3L, (r+1)*3L) */
    int32_t* pos;
    int32_t* alive;
    int64_t* stats;        /* device int64[n_steps][n_roads][8] or NULL: per step and road
                              cars (at step start), exited, moved, blocked, lost (a conflict),
                              waiting_red, spawned, lane_changes */
    uint32_t step;         /* (host) index of the next step; advanced by the call */
} abm_traffic_state;

/* Empty roads (every slot alive = 0, lane = pos = 0); sets s->step = 0. */
ABM_API int abm_traffic_init(const abm_traffic_params* p, abm_traffic_state* s, void* stream);

/* Run n_steps steps of every road from s->step, then advance s->step.  One
 * workgroup per road keeps the road in LDS for the whole call. */
ABM_API int abm_traffic_step(const abm_traffic_params* p, abm_traffic_state* s, int32_t n_steps,
                             void* stream);

/* Message describing the last non-OK status returned on this thread. */
ABM_API const char* abm_last_error(void);

/* Library version string. */
ABM_API const char* abm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ABM_H */
