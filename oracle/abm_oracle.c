/*
 * abm_oracle.c -- plain, slow, single-threaded CPU oracle for the ABMax
 * select/update hot path and the predation model built on it.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this code:
 * only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source, header, table or helper with the
 * HIP library; the two are written independently from the paper (arXiv
 * 2508.16508) and from the fixed model readings stated below.
 *
 * Everything here is integer: uint8 masks, int32 state, uint32 hashes and
 * uint64 conflict keys, so the GPU path must agree bit for bit.
 *
 * Structure:
 *   1. counter-based RNG (SplitMix64 output function, Steele/Lea/Flood 2014)
 *   2. the paper's toy task, two literal formulations (Sec. 4, Alg. 1 "Rank-
 *      Match" and Alg. 2 "Sort-Count-Iterate") -- used only to pin (3)
 *   3. primitives as plain definitions (Sec. 4 toy task; Sec. 2 API list)
 *   4. the predation model (Sec. 5.1, Fig. 2) step by step in the fixed order
 *      move, eat, breed, die, regrow
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------- */
/* 1. RNG                                                                     */
/* ------------------------------------------------------------------------- */

/* SplitMix64 output function applied to the state z: add the golden gamma,
 * then two xor-shift-multiply rounds and a final xor-shift ("Mix13" constants).
 * mix64(0) is the first SplitMix64 output from seed 0. */
ORC_API uint64_t orc_mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Counter-based draw keyed on (seed, step, agent, purpose): the high 32 bits
 * of mix64(mix64(seed:step) xor (agent:purpose)).  No state is carried, so a
 * run can be resumed from (seed, step) alone. */
ORC_API uint32_t orc_rng(uint32_t seed, uint32_t step, uint32_t agent, uint32_t purpose)
{
    uint64_t inner = orc_mix64(((uint64_t)seed << 32) | (uint64_t)step);
    uint64_t outer = orc_mix64(inner ^ (((uint64_t)agent << 32) | (uint64_t)purpose));
    return (uint32_t)(outer >> 32);
}

/* Lemire multiply-shift reduction of a 32-bit draw onto [0, n). */
ORC_API uint32_t orc_uniform(uint32_t h, uint32_t n)
{
    return (uint32_t)(((uint64_t)h * (uint64_t)n) >> 32);
}

/* ------------------------------------------------------------------------- */
/* 2. Toy task of Sec. 4: set the first r = min(p, q) even entries of a to    */
/*    the first r odd entries of b.                                           */
/* ------------------------------------------------------------------------- */

static int is_even(int64_t v) { return (v % 2) == 0; }
static int is_odd(int64_t v) { return (v % 2) != 0; }

/* Rank-Match (Sec. 4, Alg. 1).  Labels are the inclusive cumulative sum of the
 * mask multiplied by the mask (1-based for selected entries, 0 otherwise).
 * Every (a_i, b_j) pair yields a candidate: b_j when the labels agree, else
 * a_i, with an update flag; argmax over the flags (first maximum; 0 when all
 * flags are false) picks the candidate.  With guard != 0 the labels must also
 * be positive: without it an unselected a_i (label 0) matches an unselected
 * b_j (label 0) and is overwritten, which the toy task does not allow. */
ORC_API void orc_toy_rank_match(const int64_t* a, int64_t n, const int64_t* b, int64_t m,
                                int guard, int64_t* out)
{
    int64_t* ra = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    int64_t* rb = (int64_t*)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
    int64_t* cand = (int64_t*)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
    uint8_t* mu = (uint8_t*)calloc((size_t)(m > 0 ? m : 1), 1);
    int64_t cs = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t ma = is_even(a[i]);
        cs += ma;
        ra[i] = cs * ma;
    }
    cs = 0;
    for (int64_t j = 0; j < m; ++j) {
        int64_t mb = is_odd(b[j]);
        cs += mb;
        rb[j] = cs * mb;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (m == 0) { out[i] = a[i]; continue; }
        for (int64_t j = 0; j < m; ++j) {
            int match = (ra[i] == rb[j]) && (!guard || ra[i] > 0);
            cand[j] = match ? b[j] : a[i];
            mu[j] = (uint8_t)match;
        }
        int64_t best = 0; /* argmax: index of the first maximum */
        for (int64_t j = 1; j < m; ++j)
            if (mu[j] > mu[best]) best = j;
        out[i] = cand[best];
    }
    free(ra); free(rb); free(cand); free(mu);
}

/* Sort-Count-Iterate (Sec. 4, Alg. 2).  r = min(#even a, #odd b); a stable
 * ordering that puts the indices of true mask entries first; then a serial
 * loop copies b[ib[k]] into a[ia[k]] for k < r. */
ORC_API void orc_toy_sort_count_iterate(const int64_t* a, int64_t n, const int64_t* b, int64_t m,
                                        int64_t* out)
{
    int64_t* ia = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* ib = (int64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int64_t p = 0, q = 0, k = 0;
    for (int64_t i = 0; i < n; ++i) { out[i] = a[i]; p += is_even(a[i]); }
    for (int64_t j = 0; j < m; ++j) q += is_odd(b[j]);
    /* stable "trues first" ordering, written as two passes */
    for (int64_t i = 0; i < n; ++i) if (is_even(a[i])) ia[k++] = i;
    for (int64_t i = 0; i < n; ++i) if (!is_even(a[i])) ia[k++] = i;
    k = 0;
    for (int64_t j = 0; j < m; ++j) if (is_odd(b[j])) ib[k++] = j;
    for (int64_t j = 0; j < m; ++j) if (!is_odd(b[j])) ib[k++] = j;
    int64_t r = p < q ? p : q;
    for (int64_t s = 0; s < r; ++s) out[ia[s]] = b[ib[s]];
    free(ia); free(ib);
}

/* ------------------------------------------------------------------------- */
/* 3. Primitives (plain definitions).  Masks: a byte is "selected" when it is  */
/*    non-zero.  alive: a slot is live when its value is non-zero.            */
/* ------------------------------------------------------------------------- */

/* select_agents (Sec. 2): the ascending list of selected indices and its
 * length.  out_idx may be NULL to count only. */
ORC_API int64_t orc_select_indices(const uint8_t* mask, int64_t n, int64_t* out_idx)
{
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (mask[i]) {
            if (out_idx) out_idx[k] = i;
            ++k;
        }
    }
    return k;
}

/* Distinct updates to a dynamically selected subset (Sec. 4 toy task).
 * p = #selected slots, q = #selected records (all n_rec records when
 * upd_mask is NULL), r = min(p, q).  The j-th selected slot (ascending) takes
 * every attribute of the j-th selected record (ascending), for j < r.
 * Nothing else changes.  applied = r, dropped = q - r. */
ORC_API void orc_select_update(int64_t n, int32_t n_attrs, int32_t* const* attr,
                               const uint8_t* sel_mask, int64_t n_rec,
                               const int32_t* const* rec, const uint8_t* upd_mask,
                               int64_t* applied, int64_t* dropped)
{
    int64_t* A = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* B = (int64_t*)malloc((size_t)(n_rec > 0 ? n_rec : 1) * sizeof(int64_t));
    int64_t p = orc_select_indices(sel_mask, n, A);
    int64_t q;
    if (upd_mask) {
        q = orc_select_indices(upd_mask, n_rec, B);
    } else {
        q = n_rec;
        for (int64_t j = 0; j < n_rec; ++j) B[j] = j;
    }
    int64_t r = p < q ? p : q;
    for (int64_t j = 0; j < r; ++j)
        for (int32_t a = 0; a < n_attrs; ++a)
            attr[a][A[j]] = rec[a][B[j]];
    if (applied) *applied = r;
    if (dropped) *dropped = q - r;
    free(A); free(B);
}

/* add_agents: the free slots are those with alive == 0; newborn j goes to the
 * j-th lowest free slot (select_update on the free mask) and that slot becomes
 * live.  Newborns beyond the number of free slots are dropped. */
ORC_API void orc_add_agents(int64_t n, int32_t n_attrs, int32_t* const* attr, int32_t* alive,
                            int64_t n_new, const int32_t* const* rec,
                            int64_t* added, int64_t* dropped)
{
    uint8_t* freem = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
    int64_t* F = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) freem[i] = (uint8_t)(alive[i] == 0);
    int64_t nf = orc_select_indices(freem, n, F);
    int64_t r = nf < n_new ? nf : n_new;
    orc_select_update(n, n_attrs, attr, freem, n_new, rec, NULL, NULL, NULL);
    for (int64_t j = 0; j < r; ++j) alive[F[j]] = 1;
    if (added) *added = r;
    if (dropped) *dropped = n_new - r;
    free(freem); free(F);
}

/* remove_agents (set_agents_mask, Sec. 2): an independent masked update.
 * removed = #{i : kill[i] and alive[i]}; then alive[i] = 0 wherever kill[i].
 * The other fields of a removed slot are left as they were. */
ORC_API void orc_remove_agents(int64_t n, int32_t* alive, const uint8_t* kill, int64_t* removed)
{
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (kill[i]) {
            if (alive[i]) ++cnt;
            alive[i] = 0;
        }
    }
    if (removed) *removed = cnt;
}

/* Conflict resolution (Sec. 5.2: a priority per claimant of a cell).  Claim c
 * is active when active is NULL or active[c] != 0, and its target lies in
 * [0, n_targets); other claims are ignored.  key_c = prio_c * 2^32 + c.
 * best[t] = the minimum key over active claims on t (UINT64_MAX if none),
 * winner[t] = the claim index of best[t] (-1 if none),
 * won[c] = 1 exactly for the claim whose key is best[target_c]. */
ORC_API void orc_resolve_conflicts(int64_t n_claims, const int32_t* target, const uint32_t* prio,
                                   const uint8_t* active, int64_t n_targets,
                                   uint64_t* best, int32_t* winner, uint8_t* won)
{
    for (int64_t t = 0; t < n_targets; ++t) best[t] = UINT64_MAX;
    for (int64_t c = 0; c < n_claims; ++c) {
        if (active && !active[c]) continue;
        if (target[c] < 0 || (int64_t)target[c] >= n_targets) continue;
        uint64_t key = ((uint64_t)prio[c] << 32) | (uint64_t)(uint32_t)c;
        if (key < best[target[c]]) best[target[c]] = key;
    }
    for (int64_t t = 0; t < n_targets; ++t)
        winner[t] = best[t] == UINT64_MAX ? -1 : (int32_t)(uint32_t)(best[t] & 0xFFFFFFFFULL);
    for (int64_t c = 0; c < n_claims; ++c) {
        won[c] = 0;
        if (active && !active[c]) continue;
        if (target[c] < 0 || (int64_t)target[c] >= n_targets) continue;
        uint64_t key = ((uint64_t)prio[c] << 32) | (uint64_t)(uint32_t)c;
        won[c] = (uint8_t)(best[target[c]] == key);
    }
}

/* ------------------------------------------------------------------------- */
/* 4. Predation model (Sec. 5.1, Fig. 2; Wilensky's wolf-sheep-grass).         */
/* ------------------------------------------------------------------------- */

/* draw purposes */
enum {
    P_GRASS_GROWN = 0x01, P_GRASS_CD = 0x02,
    P_S_X = 0x10, P_S_Y = 0x11, P_S_E = 0x12, P_S_MOVE = 0x13,
    P_S_GRASS_KEY = 0x14, P_S_PREY_KEY = 0x15, P_S_BREED = 0x16,
    P_W_X = 0x20, P_W_Y = 0x21, P_W_E = 0x22, P_W_MOVE = 0x23,
    P_W_EAT_KEY = 0x24, P_W_BREED = 0x26
};
#define STEP_INIT 0xFFFFFFFFu

typedef struct {
    int32_t W, H;        /* toroidal lattice */
    int32_t R;           /* grass regrowth delay in steps */
    int32_t gain_s, gain_w;
    uint32_t T_s, T_w;   /* reproduction: draw < T */
    uint32_t seed;
    int64_t cap_s, cap_w; /* slot capacities */
    int64_t n_s0, n_w0;   /* initial live counts */
    int32_t multi_prey;   /* 0: one prey per cell; 1: every wolf of a cell may eat (see eat) */
} orc_pred_params;

typedef struct { int32_t *x, *y, *e, *alive; } orc_species;

typedef struct {
    int32_t* grass;       /* W*H countdown, 0 = grown; cell c = y*W + x */
    orc_species sheep, wolves;
    uint32_t step;        /* index of the next step to run */
} orc_pred_state;

typedef struct {
    int64_t live_s, live_w;       /* at the start of the step */
    int64_t grass_eaten, sheep_eaten;
    int64_t births_s, births_w;
    int64_t starved_s, starved_w;
} orc_pred_stats;

/* the eight neighbour offsets, indexed by the top three bits of a draw */
static const int32_t DX[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
static const int32_t DY[8] = {-1, -1, -1, 0, 0, 1, 1, 1};

static void init_species(const orc_pred_params* P, orc_species* s, int64_t cap, int64_t n0,
                         uint32_t px, uint32_t py, uint32_t pe, int32_t gain)
{
    for (int64_t i = 0; i < cap; ++i) {
        if (i < n0) {
            s->x[i] = (int32_t)orc_uniform(orc_rng(P->seed, STEP_INIT, (uint32_t)i, px), (uint32_t)P->W);
            s->y[i] = (int32_t)orc_uniform(orc_rng(P->seed, STEP_INIT, (uint32_t)i, py), (uint32_t)P->H);
            s->e[i] = (int32_t)orc_uniform(orc_rng(P->seed, STEP_INIT, (uint32_t)i, pe), (uint32_t)(2 * gain));
            s->alive[i] = 1;
        } else {
            s->x[i] = 0; s->y[i] = 0; s->e[i] = 0; s->alive[i] = 0;
        }
    }
}

/* Initial state: each cell is grown with probability 1/2 (draw < 2^31), else
 * it carries a countdown uniform in [1, R].  Agents occupy slots 0..n0-1 at
 * uniform cells with energy uniform in [0, 2*gain); other slots are zero. */
ORC_API void orc_predation_init(const orc_pred_params* P, orc_pred_state* S)
{
    int64_t G = (int64_t)P->W * P->H;
    for (int64_t c = 0; c < G; ++c) {
        uint32_t h = orc_rng(P->seed, STEP_INIT, (uint32_t)c, P_GRASS_GROWN);
        if (h < 0x80000000u)
            S->grass[c] = 0;
        else
            S->grass[c] = 1 + (int32_t)orc_uniform(orc_rng(P->seed, STEP_INIT, (uint32_t)c, P_GRASS_CD),
                                                   (uint32_t)P->R);
    }
    init_species(P, &S->sheep, P->cap_s, P->n_s0, P_S_X, P_S_Y, P_S_E, P->gain_s);
    init_species(P, &S->wolves, P->cap_w, P->n_w0, P_W_X, P_W_Y, P_W_E, P->gain_w);
    S->step = 0;
}

static int64_t count_live(const orc_species* s, int64_t cap)
{
    int64_t k = 0;
    for (int64_t i = 0; i < cap; ++i) k += s->alive[i] != 0;
    return k;
}

/* Phase 1: every live agent steps to one of its eight neighbours (toroidal)
 * and pays one unit of energy. */
static void move_species(const orc_pred_params* P, orc_species* s, int64_t cap, uint32_t t, uint32_t purpose)
{
    for (int64_t i = 0; i < cap; ++i) {
        if (!s->alive[i]) continue;
        uint32_t d = orc_rng(P->seed, t, (uint32_t)i, purpose) >> 29;
        s->x[i] = (s->x[i] + DX[d] + P->W) % P->W;
        s->y[i] = (s->y[i] + DY[d] + P->H) % P->H;
        s->e[i] -= 1;
    }
}

static uint64_t agent_key(uint32_t seed, uint32_t t, int64_t i, uint32_t purpose)
{
    return ((uint64_t)orc_rng(seed, t, (uint32_t)i, purpose) << 32) | (uint64_t)(uint32_t)i;
}

/* Phase 3: breeders are live agents with positive energy whose draw is below
 * T; free slots are those with alive == 0 (after eating).  The j-th breeder
 * (ascending slot) puts a child on its own cell into the j-th lowest free
 * slot; the child takes e >> 1 and the parent keeps e - (e >> 1).  Breeders
 * beyond the number of free slots are unchanged. */
static int64_t breed_species(const orc_pred_params* P, orc_species* s, int64_t cap, uint32_t t,
                             uint32_t purpose, uint32_t T)
{
    int64_t* B = (int64_t*)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(int64_t));
    int64_t* F = (int64_t*)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(int64_t));
    int64_t nb = 0, nf = 0;
    for (int64_t i = 0; i < cap; ++i) {
        if (s->alive[i] && s->e[i] > 0 && orc_rng(P->seed, t, (uint32_t)i, purpose) < T) B[nb++] = i;
        if (!s->alive[i]) F[nf++] = i;
    }
    int64_t r = nb < nf ? nb : nf;
    for (int64_t j = 0; j < r; ++j) {
        int64_t par = B[j], ch = F[j];
        int32_t ec = s->e[par] >> 1;
        s->x[ch] = s->x[par];
        s->y[ch] = s->y[par];
        s->e[ch] = ec;
        s->e[par] = s->e[par] - ec;
        s->alive[ch] = 1;
    }
    free(B); free(F);
    return r;
}

/* Phase 4: live agents with negative energy die; their other fields stay. */
static int64_t starve_species(orc_species* s, int64_t cap)
{
    int64_t k = 0;
    for (int64_t i = 0; i < cap; ++i)
        if (s->alive[i] && s->e[i] < 0) { s->alive[i] = 0; ++k; }
    return k;
}

/* The five phases of step t = S->step, exported one by one so that tests can
 * check each phase on its own; orc_predation_step runs them in order. */

/* Phase 1 for both species. */
ORC_API void orc_pred_move(const orc_pred_params* P, orc_pred_state* S)
{
    move_species(P, &S->sheep, P->cap_s, S->step, P_S_MOVE);
    move_species(P, &S->wolves, P->cap_w, S->step, P_W_MOVE);
}

/* Phase 2.  Grass first: on every grown cell holding live sheep the sheep with
 * the lowest key (draw << 32 | slot) eats it (energy += gain_s, countdown = R).
 * Then prey: on every cell holding both live sheep and live wolves, the
 * lowest-key sheep is eaten by the lowest-key wolf (energy += gain_w).  So at
 * most one grass and one sheep are consumed per cell per step. */
/* Ascending order of packed keys (the low 32 bits are the slot, so no two
 * keys of one species are equal). */
static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Prey with several matches per cell: on every cell, the live sheep are put
 * in ascending order of their prey keys and the live wolves in ascending
 * order of their eat keys, and for j < min(#sheep, #wolves) the j-th wolf
 * eats the j-th sheep (the sheep dies, the wolf gains gain_w).  With at most
 * one wolf or one sheep per cell this is the one-prey rule.  This is the
 * rank-and-match of the toy task (Sec. 4, Alg. 1) applied per cell, with
 * cells as the groups.  Returns the number of sheep eaten. */
static int64_t eat_prey_multi(const orc_pred_params* P, orc_pred_state* S)
{
    const uint32_t t = S->step;
    const int64_t G = (int64_t)P->W * P->H;
    int64_t* off_s = (int64_t*)calloc((size_t)G + 1, sizeof(int64_t));
    int64_t* off_w = (int64_t*)calloc((size_t)G + 1, sizeof(int64_t));
    int64_t* fill_s = (int64_t*)calloc((size_t)G, sizeof(int64_t));
    int64_t* fill_w = (int64_t*)calloc((size_t)G, sizeof(int64_t));
    uint64_t* ks = (uint64_t*)malloc((size_t)(P->cap_s > 0 ? P->cap_s : 1) * sizeof(uint64_t));
    uint64_t* kw = (uint64_t*)malloc((size_t)(P->cap_w > 0 ? P->cap_w : 1) * sizeof(uint64_t));
    int64_t eaten = 0;

    /* bucket the live agents of each species by cell */
    for (int64_t i = 0; i < P->cap_s; ++i)
        if (S->sheep.alive[i]) off_s[(int64_t)S->sheep.y[i] * P->W + S->sheep.x[i] + 1]++;
    for (int64_t j = 0; j < P->cap_w; ++j)
        if (S->wolves.alive[j]) off_w[(int64_t)S->wolves.y[j] * P->W + S->wolves.x[j] + 1]++;
    for (int64_t c = 0; c < G; ++c) { off_s[c + 1] += off_s[c]; off_w[c + 1] += off_w[c]; }
    for (int64_t i = 0; i < P->cap_s; ++i) {
        if (!S->sheep.alive[i]) continue;
        int64_t c = (int64_t)S->sheep.y[i] * P->W + S->sheep.x[i];
        ks[off_s[c] + fill_s[c]++] = agent_key(P->seed, t, i, P_S_PREY_KEY);
    }
    for (int64_t j = 0; j < P->cap_w; ++j) {
        if (!S->wolves.alive[j]) continue;
        int64_t c = (int64_t)S->wolves.y[j] * P->W + S->wolves.x[j];
        kw[off_w[c] + fill_w[c]++] = agent_key(P->seed, t, j, P_W_EAT_KEY);
    }
    /* per cell: order both groups by key and pair them rank by rank */
    for (int64_t c = 0; c < G; ++c) {
        int64_t n_s = off_s[c + 1] - off_s[c], n_w = off_w[c + 1] - off_w[c];
        int64_t m = n_s < n_w ? n_s : n_w;
        if (m == 0) continue;
        qsort(ks + off_s[c], (size_t)n_s, sizeof(uint64_t), cmp_u64);
        qsort(kw + off_w[c], (size_t)n_w, sizeof(uint64_t), cmp_u64);
        for (int64_t r = 0; r < m; ++r) {
            int64_t prey = (int64_t)(uint32_t)(ks[off_s[c] + r] & 0xFFFFFFFFULL);
            int64_t wolf = (int64_t)(uint32_t)(kw[off_w[c] + r] & 0xFFFFFFFFULL);
            S->sheep.alive[prey] = 0;
            S->wolves.e[wolf] += P->gain_w;
            ++eaten;
        }
    }
    free(off_s); free(off_w); free(fill_s); free(fill_w); free(ks); free(kw);
    return eaten;
}

ORC_API void orc_pred_eat(const orc_pred_params* P, orc_pred_state* S,
                          int64_t* grass_eaten, int64_t* sheep_eaten)
{
    const uint32_t t = S->step;
    const int64_t G = (int64_t)P->W * P->H;
    uint64_t* best = (uint64_t*)malloc((size_t)G * sizeof(uint64_t));
    uint64_t* best2 = (uint64_t*)malloc((size_t)G * sizeof(uint64_t));
    int64_t ng = 0, ns = 0;

    for (int64_t c = 0; c < G; ++c) best[c] = UINT64_MAX;
    for (int64_t i = 0; i < P->cap_s; ++i) {
        if (!S->sheep.alive[i]) continue;
        int64_t c = (int64_t)S->sheep.y[i] * P->W + S->sheep.x[i];
        if (S->grass[c] != 0) continue;
        uint64_t k = agent_key(P->seed, t, i, P_S_GRASS_KEY);
        if (k < best[c]) best[c] = k;
    }
    for (int64_t c = 0; c < G; ++c) {
        if (best[c] == UINT64_MAX) continue;
        int64_t w = (int64_t)(uint32_t)(best[c] & 0xFFFFFFFFULL);
        S->sheep.e[w] += P->gain_s;
        S->grass[c] = P->R;
        ++ng;
    }

    if (P->multi_prey) {
        free(best); free(best2);
        ns = eat_prey_multi(P, S);
        if (grass_eaten) *grass_eaten = ng;
        if (sheep_eaten) *sheep_eaten = ns;
        return;
    }
    for (int64_t c = 0; c < G; ++c) { best[c] = UINT64_MAX; best2[c] = UINT64_MAX; }
    for (int64_t i = 0; i < P->cap_s; ++i) {
        if (!S->sheep.alive[i]) continue;
        int64_t c = (int64_t)S->sheep.y[i] * P->W + S->sheep.x[i];
        uint64_t k = agent_key(P->seed, t, i, P_S_PREY_KEY);
        if (k < best[c]) best[c] = k;
    }
    for (int64_t j = 0; j < P->cap_w; ++j) {
        if (!S->wolves.alive[j]) continue;
        int64_t c = (int64_t)S->wolves.y[j] * P->W + S->wolves.x[j];
        uint64_t k = agent_key(P->seed, t, j, P_W_EAT_KEY);
        if (k < best2[c]) best2[c] = k;
    }
    for (int64_t c = 0; c < G; ++c) {
        if (best[c] == UINT64_MAX || best2[c] == UINT64_MAX) continue;
        int64_t prey = (int64_t)(uint32_t)(best[c] & 0xFFFFFFFFULL);
        int64_t wolf = (int64_t)(uint32_t)(best2[c] & 0xFFFFFFFFULL);
        S->sheep.alive[prey] = 0;
        S->wolves.e[wolf] += P->gain_w;
        ++ns;
    }
    free(best); free(best2);
    if (grass_eaten) *grass_eaten = ng;
    if (sheep_eaten) *sheep_eaten = ns;
}

/* Phase 3 for both species. */
ORC_API void orc_pred_breed(const orc_pred_params* P, orc_pred_state* S,
                            int64_t* births_s, int64_t* births_w)
{
    int64_t bs = breed_species(P, &S->sheep, P->cap_s, S->step, P_S_BREED, P->T_s);
    int64_t bw = breed_species(P, &S->wolves, P->cap_w, S->step, P_W_BREED, P->T_w);
    if (births_s) *births_s = bs;
    if (births_w) *births_w = bw;
}

/* Phase 4 for both species. */
ORC_API void orc_pred_die(const orc_pred_params* P, orc_pred_state* S,
                          int64_t* starved_s, int64_t* starved_w)
{
    int64_t ss = starve_species(&S->sheep, P->cap_s);
    int64_t sw = starve_species(&S->wolves, P->cap_w);
    if (starved_s) *starved_s = ss;
    if (starved_w) *starved_w = sw;
}

/* Phase 5: every countdown above zero drops by one, so a cell eaten at step t
 * is grown again at step t + R. */
ORC_API void orc_pred_regrow(const orc_pred_params* P, orc_pred_state* S)
{
    const int64_t G = (int64_t)P->W * P->H;
    for (int64_t c = 0; c < G; ++c)
        if (S->grass[c] > 0) S->grass[c] -= 1;
}

/* One step t = S->step in the order move, eat, breed, die, regrow; then the
 * step counter advances.  Statistics of the step go to *st when given. */
ORC_API void orc_predation_step(const orc_pred_params* P, orc_pred_state* S, orc_pred_stats* st)
{
    orc_pred_stats loc;
    memset(&loc, 0, sizeof loc);
    loc.live_s = count_live(&S->sheep, P->cap_s);
    loc.live_w = count_live(&S->wolves, P->cap_w);
    orc_pred_move(P, S);
    orc_pred_eat(P, S, &loc.grass_eaten, &loc.sheep_eaten);
    orc_pred_breed(P, S, &loc.births_s, &loc.births_w);
    orc_pred_die(P, S, &loc.starved_s, &loc.starved_w);
    orc_pred_regrow(P, S);
    S->step += 1;
    if (st) *st = loc;
}

/* Run n_steps steps; per-step statistics go to stats[0..n_steps) if given. */
ORC_API void orc_predation_run(const orc_pred_params* P, orc_pred_state* S, int32_t n_steps,
                               orc_pred_stats* stats)
{
    for (int32_t k = 0; k < n_steps; ++k)
        orc_predation_step(P, S, stats ? &stats[k] : NULL);
}

/* ------------------------------------------------------------------------- */
/* 5. Traffic cellular automaton (Sec. 5.2, Fig. 4).                           */
/*                                                                           */
/* A road of 3 lanes x L cells; cell (lane, x), x = 0 the entry column and     */
/* x = L-1 the exit column.  Cars are agents in 3L slots with attributes lane,  */
/* pos and alive.  The paper fixes the ingredients (entry cells, exit cells     */
/* under signals, random lane changes, one car per cell, conflicts resolved by  */
/* cells acting as agents with a priority mask over their incoming directions,  */
/* spawning into free entry cells) but no numbers; the rules below are the      */
/* reading used here.  Step t:                                                 */
/*   1. lights: exit lane l is green iff draw(t, l, LIGHT) < T_green;          */
/*   2. every car decides on the occupancy at the start of the step: a car in  */
/*      the exit column leaves if its light is green and waits otherwise; any */
/*      other car picks left / straight / right uniformly (Lemire reduction of */
/*      draw(t, slot, LANE) onto 3; a lane off the road means straight) and    */
/*      claims the cell one column ahead in that lane, unless it is occupied  */
/*      (then it waits);                                                      */
/*   3. each claimed cell admits one claimant: the one arriving straight, else */
/*      the one from the lane below, else the one from the lane above (the     */
/*      cell's priority mask; resolve_conflicts with those priorities);       */
/*      winners move, the others wait;                                        */
/*   4. leaving cars are removed (remove_agents);                             */
/*   5. every entry cell l that is free now spawns a car if draw(t, l, SPAWN) */
/*      < T_spawn; the spawned cars, in lane order, go to the lowest free     */
/*      slots (add_agents).                                                    */
/* ------------------------------------------------------------------------- */

enum { P_T_LIGHT = 0x30, P_T_LANE = 0x31, P_T_SPAWN = 0x32 };

typedef struct {
    int32_t length;           /* cells per lane, >= 2 */
    uint32_t T_green, T_spawn;
    uint32_t seed;
} orc_traffic_params;

typedef struct {
    int32_t *lane, *pos, *alive;   /* [3 * length] car slots */
    uint32_t step;
} orc_traffic_state;

typedef struct {
    int64_t cars;          /* at the start of the step */
    int64_t exited, moved, blocked, lost, waiting_red, spawned;
    int64_t lane_changes;
} orc_traffic_stats;

ORC_API void orc_traffic_init(const orc_traffic_params* P, orc_traffic_state* S)
{
    for (int64_t i = 0; i < 3 * (int64_t)P->length; ++i) {
        S->lane[i] = 0; S->pos[i] = 0; S->alive[i] = 0;
    }
    S->step = 0;
}

ORC_API void orc_traffic_step(const orc_traffic_params* P, orc_traffic_state* S,
                              orc_traffic_stats* st)
{
    const int64_t L = P->length, n = 3 * L;
    const uint32_t t = S->step;
    orc_traffic_stats loc;
    memset(&loc, 0, sizeof loc);
    int32_t* occ = (int32_t*)malloc((size_t)n * sizeof(int32_t));      /* cell -> slot or -1 */
    int32_t* target = (int32_t*)malloc((size_t)n * sizeof(int32_t));   /* slot -> claimed cell */
    uint32_t* prio = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
    uint8_t* active = (uint8_t*)malloc((size_t)n);
    uint8_t* leave = (uint8_t*)malloc((size_t)n);
    uint64_t* best = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
    int32_t* winner = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    uint8_t* won = (uint8_t*)malloc((size_t)n);
    int green[3];

    for (int64_t c = 0; c < n; ++c) occ[c] = -1;
    for (int64_t i = 0; i < n; ++i)
        if (S->alive[i]) { occ[(int64_t)S->lane[i] * L + S->pos[i]] = (int32_t)i; loc.cars++; }
    for (int l = 0; l < 3; ++l) green[l] = orc_rng(P->seed, t, (uint32_t)l, P_T_LIGHT) < P->T_green;

    /* 2. decisions on the start-of-step occupancy */
    for (int64_t i = 0; i < n; ++i) {
        active[i] = 0; leave[i] = 0; target[i] = -1; prio[i] = 0;
        if (!S->alive[i]) continue;
        const int32_t l = S->lane[i], x = S->pos[i];
        if (x == L - 1) {
            if (green[l]) leave[i] = 1; else loc.waiting_red++;
            continue;
        }
        int32_t dl = (int32_t)orc_uniform(orc_rng(P->seed, t, (uint32_t)i, P_T_LANE), 3u) - 1;
        int32_t nl = l + dl;
        if (nl < 0 || nl > 2) nl = l;
        const int64_t c = (int64_t)nl * L + (x + 1);
        if (occ[c] >= 0) { loc.blocked++; continue; }
        target[i] = (int32_t)c;
        active[i] = 1;
        /* the target cell's priority over its three incoming directions */
        prio[i] = nl == l ? 0u : (l < nl ? 1u : 2u);
    }
    /* 3. one claimant per cell */
    orc_resolve_conflicts(n, target, prio, active, n, best, winner, won);
    for (int64_t i = 0; i < n; ++i) {
        if (!active[i]) continue;
        if (won[i]) {
            const int32_t nl = target[i] / (int32_t)L;
            if (nl != S->lane[i]) loc.lane_changes++;
            S->lane[i] = nl;
            S->pos[i] = target[i] % (int32_t)L;
            loc.moved++;
        } else {
            loc.lost++;
        }
    }
    /* 4. exits */
    {
        int64_t removed = 0;
        orc_remove_agents(n, S->alive, leave, &removed);
        loc.exited = removed;
    }
    /* 5. spawning into free entry cells */
    {
        int32_t free_entry[3] = {1, 1, 1};
        for (int64_t i = 0; i < n; ++i)
            if (S->alive[i] && S->pos[i] == 0) free_entry[S->lane[i]] = 0;
        int32_t rec_lane[3], rec_pos[3];
        int64_t q = 0;
        for (int l = 0; l < 3; ++l)
            if (free_entry[l] && orc_rng(P->seed, t, (uint32_t)l, P_T_SPAWN) < P->T_spawn) {
                rec_lane[q] = l; rec_pos[q] = 0; ++q;
            }
        int32_t* attr[2] = {S->lane, S->pos};
        const int32_t* rec[2] = {rec_lane, rec_pos};
        int64_t added = 0, dropped = 0;
        orc_add_agents(n, 2, attr, S->alive, q, rec, &added, &dropped);
        loc.spawned = added;
    }
    free(occ); free(target); free(prio); free(active); free(leave);
    free(best); free(winner); free(won);
    S->step += 1;
    if (st) *st = loc;
}

ORC_API void orc_traffic_run(const orc_traffic_params* P, orc_traffic_state* S, int32_t n_steps,
                             orc_traffic_stats* stats)
{
    for (int32_t k = 0; k < n_steps; ++k) orc_traffic_step(P, S, stats ? &stats[k] : NULL);
}

/* ------------------------------------------------------------------------- */
/* 6. sort_agents and select_agents (Sec. 2 API list).                         */
/* ------------------------------------------------------------------------- */

typedef struct { int32_t key; int64_t idx; } key_idx;

static int cmp_key_asc(const void* a, const void* b)
{
    const key_idx* x = (const key_idx*)a;
    const key_idx* y = (const key_idx*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

static int cmp_key_desc(const void* a, const void* b)
{
    const key_idx* x = (const key_idx*)a;
    const key_idx* y = (const key_idx*)b;
    if (x->key != y->key) return x->key > y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

/* sort_agents: reorder every attribute of the collection by the runtime key
 * (one int32 per agent), ascending or descending; agents with equal keys keep
 * their index order (a stable sort).  perm[j] = the old index of the agent now
 * at position j (may be NULL).  alive, if given, is reordered like the
 * attributes. */
ORC_API void orc_sort_agents(int64_t n, int32_t n_attrs, int32_t* const* attr, int32_t* alive,
                             const int32_t* key, int32_t descending, int32_t* perm)
{
    key_idx* ki = (key_idx*)malloc((size_t)(n > 0 ? n : 1) * sizeof(key_idx));
    int32_t* tmp = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) { ki[i].key = key[i]; ki[i].idx = i; }
    qsort(ki, (size_t)n, sizeof(key_idx), descending ? cmp_key_desc : cmp_key_asc);
    for (int32_t a = -1; a < n_attrs; ++a) {
        int32_t* col = a < 0 ? alive : attr[a];
        if (!col) continue;
        for (int64_t j = 0; j < n; ++j) tmp[j] = col[ki[j].idx];
        memcpy(col, tmp, (size_t)n * sizeof(int32_t));
    }
    if (perm)
        for (int64_t j = 0; j < n; ++j) perm[j] = (int32_t)ki[j].idx;
    free(ki); free(tmp);
}

/* select_agents: the indices of the agents that satisfy the condition, in
 * index order, then the others, in index order; returns how many satisfy it. */
ORC_API int64_t orc_select_agents(const uint8_t* cond, int64_t n, int32_t* order)
{
    int64_t p = 0;
    for (int64_t i = 0; i < n; ++i)
        if (cond[i]) order[p++] = (int32_t)i;
    int64_t q = p;
    for (int64_t i = 0; i < n; ++i)
        if (!cond[i]) order[q++] = (int32_t)i;
    return p;
}

/* ------------------------------------------------------------------------- */
/* 7. Limit order books with batch matching (Sec. 5.3, Fig. 5).                */
/*                                                                           */
/* Each book holds up to `cap` orders (agents: side, price, qty, time, alive)  */
/* and a last price.  Step t of a book (draws keyed on (seed, t, trader,       */
/* purpose)):                                                                 */
/*   1. expiry: orders placed E or more steps ago are cancelled;              */
/*   2. orders: trader k (0..K-1) places an order when draw(k, ORDER) <       */
/*      T_order: a buy when draw(k, SIDE) < 2^31, else a sell, at price       */
/*      last + u - D with u uniform on [0, 2D] (clamped to [1, 2^24 - 1]), for */
/*      1 + (uniform on [0, Q)) shares; the new orders, in trader order, take */
/*      the lowest free slots (add_agents); the ones that find none are       */
/*      dropped;                                                               */
/*   3. matching: buys in price-time priority (price descending, then time,  */
/*      then slot), sells likewise with price ascending; CB and CS are the    */
/*      cumulative shares along those lists; the matched volume is            */
/*      V = max over buys r of min(CB_r, CS(p_r)), CS(p) = shares of the      */
/*      sells priced at most p; the r-th buy fills clamp(V - CB_{r-1}, 0,     */
/*      q_r) and each sell likewise; the new last price is the floor of the   */
/*      mean of the buy price and the sell price covering share V;            */
/*   4. filled orders are removed, partly filled ones keep the rest.          */
/* ------------------------------------------------------------------------- */

enum { P_L_ORDER = 0x40, P_L_SIDE = 0x41, P_L_PRICE = 0x42, P_L_QTY = 0x43 };
#define LOB_MAX_PRICE ((1 << 24) - 1)

typedef struct {
    int32_t cap;           /* order slots per book */
    int32_t traders;       /* K */
    uint32_t T_order;      /* a trader orders when its draw < T_order */
    int32_t spread;        /* D: price offsets on [-D, D] ticks */
    int32_t max_qty;       /* Q: quantities on [1, Q] */
    int32_t expiry;        /* E: an order lives E steps */
    int32_t price0;        /* initial last price */
    uint32_t seed;
} orc_lob_params;

typedef struct {
    int32_t *side, *price, *qty, *time, *alive;   /* [cap]; side 0 buy, 1 sell */
    int32_t last_price;
    uint32_t step;
} orc_lob_state;

typedef struct {
    int64_t buys, sells;      /* active after matching */
    int64_t placed, dropped, expired;
    int64_t volume, filled_orders;
    int64_t price;
} orc_lob_stats;

ORC_API void orc_lob_init(const orc_lob_params* P, orc_lob_state* S)
{
    for (int32_t i = 0; i < P->cap; ++i) {
        S->side[i] = 0; S->price[i] = 0; S->qty[i] = 0; S->time[i] = 0; S->alive[i] = 0;
    }
    S->last_price = P->price0;
    S->step = 0;
}

/* price-time priority: does order a come before order b (same side)? */
static int lob_before(const orc_lob_state* S, int32_t a, int32_t b)
{
    if (S->price[a] != S->price[b])
        return S->side[a] == 0 ? S->price[a] > S->price[b] : S->price[a] < S->price[b];
    if (S->time[a] != S->time[b]) return S->time[a] < S->time[b];
    return a < b;
}

static const orc_lob_state* g_lob_sort_state;
static int cmp_lob(const void* x, const void* y)
{
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    if (a == b) return 0;
    return lob_before(g_lob_sort_state, a, b) ? -1 : 1;
}

ORC_API void orc_lob_step(const orc_lob_params* P, orc_lob_state* S, orc_lob_stats* st)
{
    const int32_t C = P->cap;
    const uint32_t t = S->step;
    orc_lob_stats loc;
    memset(&loc, 0, sizeof loc);
    uint8_t* kill = (uint8_t*)calloc((size_t)C, 1);
    int32_t* buy = (int32_t*)malloc((size_t)C * sizeof(int32_t));
    int32_t* sell = (int32_t*)malloc((size_t)C * sizeof(int32_t));
    int64_t* cb = (int64_t*)malloc(((size_t)C + 1) * sizeof(int64_t));
    int64_t* cs = (int64_t*)malloc(((size_t)C + 1) * sizeof(int64_t));

    /* 1. expiry */
    for (int32_t i = 0; i < C; ++i)
        kill[i] = (uint8_t)(S->alive[i] && (int64_t)t - S->time[i] >= P->expiry);
    orc_remove_agents(C, S->alive, kill, &loc.expired);

    /* 2. new orders, in trader order, into the lowest free slots */
    {
        int32_t* rs = (int32_t*)malloc((size_t)(P->traders > 0 ? P->traders : 1) * 4 * sizeof(int32_t));
        int32_t *r_side = rs, *r_price = rs + P->traders, *r_qty = rs + 2 * P->traders,
                *r_time = rs + 3 * P->traders;
        int64_t q = 0;
        for (int32_t k = 0; k < P->traders; ++k) {
            if (orc_rng(P->seed, t, (uint32_t)k, P_L_ORDER) >= P->T_order) continue;
            int64_t price = (int64_t)S->last_price - P->spread +
                            orc_uniform(orc_rng(P->seed, t, (uint32_t)k, P_L_PRICE),
                                        (uint32_t)(2 * P->spread + 1));
            if (price < 1) price = 1;
            if (price > LOB_MAX_PRICE) price = LOB_MAX_PRICE;
            r_side[q] = orc_rng(P->seed, t, (uint32_t)k, P_L_SIDE) < 0x80000000u ? 0 : 1;
            r_price[q] = (int32_t)price;
            r_qty[q] = 1 + (int32_t)orc_uniform(orc_rng(P->seed, t, (uint32_t)k, P_L_QTY),
                                               (uint32_t)P->max_qty);
            r_time[q] = (int32_t)t;
            ++q;
        }
        int32_t* attr[4] = {S->side, S->price, S->qty, S->time};
        const int32_t* rec[4] = {r_side, r_price, r_qty, r_time};
        int64_t added = 0, dropped = 0;
        orc_add_agents(C, 4, attr, S->alive, q, rec, &added, &dropped);
        loc.placed = added;
        loc.dropped = dropped;
        free(rs);
    }

    /* 3. batch matching: both sides in priority order, cumulative shares */
    int64_t nb = 0, ns = 0;
    for (int32_t i = 0; i < C; ++i) {
        if (!S->alive[i]) continue;
        if (S->side[i] == 0) buy[nb++] = i; else sell[ns++] = i;
    }
    g_lob_sort_state = S;
    qsort(buy, (size_t)nb, sizeof(int32_t), cmp_lob);
    qsort(sell, (size_t)ns, sizeof(int32_t), cmp_lob);
    cb[0] = 0; cs[0] = 0;
    for (int64_t r = 0; r < nb; ++r) cb[r + 1] = cb[r] + S->qty[buy[r]];
    for (int64_t r = 0; r < ns; ++r) cs[r + 1] = cs[r] + S->qty[sell[r]];
    int64_t V = 0;
    for (int64_t r = 0; r < nb; ++r) {
        int64_t m = 0;                       /* sells priced at most the buy's price */
        while (m < ns && S->price[sell[m]] <= S->price[buy[r]]) ++m;
        int64_t v = cb[r + 1] < cs[m] ? cb[r + 1] : cs[m];
        if (v > V) V = v;
    }
    loc.volume = V;
    if (V > 0) {
        int64_t rb = 0, rsl = 0;             /* the orders covering share V */
        while (cb[rb + 1] < V) ++rb;
        while (cs[rsl + 1] < V) ++rsl;
        S->last_price = (int32_t)(((int64_t)S->price[buy[rb]] + S->price[sell[rsl]]) / 2);
    }
    /* 4. fills */
    for (int i = 0; i < C; ++i) kill[i] = 0;
    for (int s = 0; s < 2; ++s) {
        const int64_t n = s ? ns : nb;
        const int32_t* list = s ? sell : buy;
        const int64_t* cum = s ? cs : cb;
        for (int64_t r = 0; r < n; ++r) {
            int64_t f = V - cum[r];
            if (f <= 0) break;
            const int32_t i = list[r];
            if (f >= S->qty[i]) { kill[i] = 1; f = S->qty[i]; }
            else S->qty[i] -= (int32_t)f;
            loc.filled_orders++;
        }
    }
    {
        int64_t removed = 0;
        orc_remove_agents(C, S->alive, kill, &removed);
    }
    for (int32_t i = 0; i < C; ++i) {
        if (!S->alive[i]) continue;
        if (S->side[i] == 0) loc.buys++; else loc.sells++;
    }
    loc.price = S->last_price;
    free(kill); free(buy); free(sell); free(cb); free(cs);
    S->step += 1;
    if (st) *st = loc;
}
