/*
 * hgoracle.c -- plain, single-threaded CPU oracle for the km1 label-propagation
 * refinement core of "Scalable Shared-Memory Hypergraph Partitioning"
 * (Gottesbueren, Heuer, Sanders, Schlag; arXiv 2010.10272).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) may link, import or call this file.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * Every function below is the textbook definition written out, or the
 * synchronous LP round taken step by step, with no blocking, fusion or
 * incremental bookkeeping.  Pin counts, connectivity and block weights are
 * recomputed from scratch from the partition whenever they are needed.  All
 * arithmetic is integer (int32 ids and weights, int64 sums); the only floating
 * point is the one double product that turns epsilon into L_max.
 *
 * Notation follows the paper (section "Preliminaries"):
 *   H = (V, E, c, w): n vertices, m nets, vertex weights c, net weights w.
 *   Net e is a set of pins; I(v) is the set of nets incident to v.
 *   Pi: V -> {0..k-1} (blocks are 0-based here; the paper counts from 1).
 *   Phi(e,i) = |e intersect V_i|, Lambda(e) = {i : Phi(e,i) > 0},
 *   lambda(e) = |Lambda(e)|, km1 = sum_e (lambda(e)-1) w(e).
 *
 * Readings of points the paper leaves open (tie-break, approval order, ...)
 * are listed where they are used and collected in the design notes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_INVALID (-1)
#define OR_ERR_UNSUPPORTED (-2)

typedef struct {
  int64_t eligible;       /* |E_r|: vertices eligible at round start          */
  int64_t boundary;       /* |A_r|: eligible vertices that are boundary       */
  int64_t candidates;     /* vertices whose best move passes the move rule    */
  int64_t approved;       /* moves approved against L_max (= moves applied)   */
  int64_t moved_pins;     /* sum of d(u) over moved u                         */
  int64_t touched_nets;   /* nets holding at least one moved vertex           */
  int64_t km1_delta;      /* km1(before) - km1(after), both recomputed        */
  int64_t km1_after;      /* km1 after the round                              */
  int64_t max_block_weight; /* max_i c(V_i) after the round                   */
  int64_t active_pins;    /* sum of d(u) over active (eligible boundary) u    */
  int64_t touched_pins;   /* sum of |e| over the touched nets                 */
} or_round_stats;

/* ------------------------------------------------------------------------ */
/* Input checks (section "Preliminaries": nets are non-empty vertex subsets, */
/* weights are positive).                                                    */
/* ------------------------------------------------------------------------ */

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Returns OR_OK if (eptr, pins, c, w) is a valid weighted hypergraph:
 * eptr[0] = 0, eptr[m] = P, every net non-empty, pins in [0,n), no vertex twice
 * in one net (a net is a set), all weights > 0.  c or w may be NULL (unit). */
int or_check_hypergraph(int32_t n, int32_t m, int64_t P, const int64_t* eptr,
                        const int32_t* pins, const int32_t* c, const int32_t* w) {
  if (n < 1 || m < 1 || P < m) return OR_ERR_INVALID;
  if (eptr[0] != 0 || eptr[m] != P) return OR_ERR_INVALID;
  int64_t maxlen = 0;
  for (int32_t e = 0; e < m; ++e) {
    if (eptr[e + 1] <= eptr[e]) return OR_ERR_INVALID; /* empty net */
    if (eptr[e + 1] - eptr[e] > maxlen) maxlen = eptr[e + 1] - eptr[e];
  }
  for (int64_t p = 0; p < P; ++p)
    if (pins[p] < 0 || pins[p] >= n) return OR_ERR_INVALID;
  int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)maxlen);
  if (!tmp) return OR_ERR_INVALID;
  int bad = 0;
  for (int32_t e = 0; e < m && !bad; ++e) {
    int64_t len = eptr[e + 1] - eptr[e];
    memcpy(tmp, pins + eptr[e], sizeof(int32_t) * (size_t)len);
    qsort(tmp, (size_t)len, sizeof(int32_t), cmp_i32);
    for (int64_t j = 1; j < len; ++j)
      if (tmp[j] == tmp[j - 1]) { bad = 1; break; }
  }
  free(tmp);
  if (bad) return OR_ERR_INVALID;
  if (c) for (int32_t v = 0; v < n; ++v) if (c[v] <= 0) return OR_ERR_INVALID;
  if (w) for (int32_t e = 0; e < m; ++e) if (w[e] <= 0) return OR_ERR_INVALID;
  return OR_OK;
}

int or_check_partition(int32_t n, const int32_t* part, int32_t k) {
  if (k < 2) return OR_ERR_INVALID;
  for (int32_t v = 0; v < n; ++v)
    if (part[v] < 0 || part[v] >= k) return OR_ERR_INVALID;
  return OR_OK;
}

static inline int64_t cw(const int32_t* c, int32_t v) { return c ? (int64_t)c[v] : 1; }
static inline int64_t ww(const int32_t* w, int32_t e) { return w ? (int64_t)w[e] : 1; }

/* ------------------------------------------------------------------------ */
/* Incident nets I(v), listed in increasing net id.                          */
/* ------------------------------------------------------------------------ */
void or_incidence(int32_t n, int32_t m, const int64_t* eptr, const int32_t* pins,
                  int64_t* vptr, int32_t* vnets) {
  for (int32_t v = 0; v <= n; ++v) vptr[v] = 0;
  for (int32_t e = 0; e < m; ++e)
    for (int64_t p = eptr[e]; p < eptr[e + 1]; ++p) vptr[pins[p] + 1] += 1;
  for (int32_t v = 0; v < n; ++v) vptr[v + 1] += vptr[v];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  for (int32_t v = 0; v < n; ++v) fill[v] = vptr[v];
  for (int32_t e = 0; e < m; ++e) /* nets in increasing id => rows sorted */
    for (int64_t p = eptr[e]; p < eptr[e + 1]; ++p) vnets[fill[pins[p]]++] = e;
  free(fill);
}

/* ------------------------------------------------------------------------ */
/* Pin counts Phi(e,i) = |{v in e : Pi(v) = i}|   (section "Preliminaries")  */
/* ------------------------------------------------------------------------ */
void or_pin_counts(int32_t m, const int64_t* eptr, const int32_t* pins,
                   const int32_t* part, int32_t k, int32_t* phi) {
  memset(phi, 0, sizeof(int32_t) * (size_t)m * (size_t)k);
  for (int32_t e = 0; e < m; ++e)
    for (int64_t p = eptr[e]; p < eptr[e + 1]; ++p)
      phi[(int64_t)e * k + part[pins[p]]] += 1;
}

/* Connectivity set Lambda(e) = {i : Phi(e,i) > 0} as a bitset of ceil(k/32)
 * words (bit i%32 of word i/32), and connectivity lambda(e) = |Lambda(e)|. */
void or_connectivity(int32_t m, int32_t k, const int32_t* phi, int32_t* lambda,
                     uint32_t* conn) {
  int32_t wk = (k + 31) / 32;
  for (int32_t e = 0; e < m; ++e) {
    int32_t l = 0;
    for (int32_t j = 0; j < wk; ++j) conn[(int64_t)e * wk + j] = 0;
    for (int32_t i = 0; i < k; ++i) {
      if (phi[(int64_t)e * k + i] > 0) {
        l += 1;
        conn[(int64_t)e * wk + i / 32] |= (uint32_t)1 << (i % 32);
      }
    }
    lambda[e] = l;
  }
}

/* Block weights c(V_i) = sum of c(v) over v with Pi(v) = i. */
void or_block_weights(int32_t n, const int32_t* c, const int32_t* part, int32_t k,
                      int64_t* W) {
  for (int32_t i = 0; i < k; ++i) W[i] = 0;
  for (int32_t v = 0; v < n; ++v) W[part[v]] += cw(c, v);
}

/* Connectivity metric (lambda - 1)(Pi) = sum_e (lambda(e) - 1) w(e). */
int64_t or_km1(int32_t m, const int32_t* w, const int32_t* lambda) {
  int64_t s = 0;
  for (int32_t e = 0; e < m; ++e) s += (int64_t)(lambda[e] - 1) * ww(w, e);
  return s;
}

/* L_max = (1 + eps) * ceil(c(V) / k) (section "Preliminaries").  Block weights
 * are integers, so c(V_i) <= L_max is the same as c(V_i) <= floor(L_max). */
int64_t or_lmax(int64_t total_weight, int32_t k, double eps) {
  int64_t avg = (total_weight + k - 1) / k;
  return (int64_t)floor((1.0 + eps) * (double)avg);
}

/* ------------------------------------------------------------------------ */
/* Gains (section "Parallel Gain Calculation"):                              */
/*   b(u)   = w({e in I(u) : Phi(e, Pi(u)) = 1})                             */
/*   p_i(u) = w({e in I(u) : Phi(e, V_i)  = 0})                              */
/*   g_i(u) = b(u) - p_i(u)  for i != Pi(u);  g_{Pi(u)}(u) = 0 (moving a     */
/*   vertex into its own block changes nothing).                             */
/* gains: n*k row-major; benefit: n entries or NULL.                         */
/* ------------------------------------------------------------------------ */
void or_gains(int32_t n, const int64_t* vptr, const int32_t* vnets, const int32_t* w,
              const int32_t* part, int32_t k, const int32_t* phi, int64_t* gains,
              int64_t* benefit) {
  int64_t* p = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  for (int32_t u = 0; u < n; ++u) {
    int32_t a = part[u];
    int64_t b = 0;
    for (int32_t i = 0; i < k; ++i) p[i] = 0;
    for (int64_t j = vptr[u]; j < vptr[u + 1]; ++j) {
      int32_t e = vnets[j];
      if (phi[(int64_t)e * k + a] == 1) b += ww(w, e);
      for (int32_t i = 0; i < k; ++i)
        if (phi[(int64_t)e * k + i] == 0) p[i] += ww(w, e);
    }
    for (int32_t i = 0; i < k; ++i)
      gains[(int64_t)u * k + i] = (i == a) ? 0 : b - p[i];
    if (benefit) benefit[u] = b;
  }
  free(p);
}

/* ------------------------------------------------------------------------ */
/* Gain cache contents (subsection "Gain Caching"): the terms kept apart so  */
/* that a gain is b(u) - p_i(u), for every vertex u                          */
/*   benefit[u]    = b(u)   = w({e in I(u) : Phi(e, Pi(u)) = 1})             */
/*   incident[u]   = w(I(u))                                                 */
/*   penalty[u*k+i]= p_i(u) = w({e in I(u) : Phi(e, i) = 0})   (all i,       */
/*                   so p_{Pi(u)}(u) = 0)                                    */
/* ------------------------------------------------------------------------ */
void or_gain_cache(int32_t n, const int64_t* vptr, const int32_t* vnets, const int32_t* w,
                   const int32_t* part, int32_t k, const int32_t* phi, int64_t* benefit,
                   int64_t* incident, int64_t* penalty) {
  for (int32_t u = 0; u < n; ++u) {
    int32_t a = part[u];
    int64_t b = 0, tot = 0;
    int64_t* p = penalty + (int64_t)u * k;
    for (int32_t i = 0; i < k; ++i) p[i] = 0;
    for (int64_t j = vptr[u]; j < vptr[u + 1]; ++j) {
      int32_t e = vnets[j];
      tot += ww(w, e);
      if (phi[(int64_t)e * k + a] == 1) b += ww(w, e);
      for (int32_t i = 0; i < k; ++i)
        if (phi[(int64_t)e * k + i] == 0) p[i] += ww(w, e);
    }
    benefit[u] = b;
    incident[u] = tot;
  }
}

/* ------------------------------------------------------------------------ */
/* One synchronous label-propagation round (section "Label Propagation"),   */
/* re-specified for synchronous execution:                                   */
/*  1. eligible set E (given), active set A = eligible boundary vertices;    */
/*  2. for u in A: neighbouring blocks T(u) = union of Lambda(e) over I(u)   */
/*     minus Pi(u); feasible F(u) = {i in T(u): c(V_i) + c(u) <= L_max};     */
/*     best target by (gain desc, c(V_i) asc, i asc);                         */
/*  3. u is a candidate if that gain is > 0, or = 0 and the move makes the    */
/*     heavier side lighter: c(V_t) + c(u) < c(V_Pi(u));                      */
/*  4. approval per target block t: candidates sorted by (gain desc, id asc),*/
/*     the longest prefix whose weight fits c(V_t) + prefix <= L_max;         */
/*  5. all approved moves are applied at once; Phi/lambda/c(V_i) are then    */
/*     recomputed from scratch; the next eligible set is every pin of every  */
/*     net that holds a moved vertex.                                         */
/* All decisions read the round-start state only.                            */
/* ------------------------------------------------------------------------ */

typedef struct { int64_t gain; int32_t u; int32_t t; } or_cand;

static int cmp_cand(const void* x, const void* y) {
  const or_cand* a = (const or_cand*)x;
  const or_cand* b = (const or_cand*)y;
  if (a->t != b->t) return (a->t > b->t) - (a->t < b->t);
  if (a->gain != b->gain) return (a->gain < b->gain) - (a->gain > b->gain); /* desc */
  return (a->u > b->u) - (a->u < b->u);
}

/* (gain desc, id asc): the order of a round's moves for exact gains */
static int cmp_gain_id(const void* x, const void* y) {
  const or_cand* a = (const or_cand*)x;
  const or_cand* b = (const or_cand*)y;
  if (a->gain != b->gain) return (a->gain < b->gain) - (a->gain > b->gain); /* desc */
  return (a->u > b->u) - (a->u < b->u);
}

static int lp_round_impl(int32_t n, int32_t m, const int64_t* eptr, const int32_t* pins,
                         const int64_t* vptr, const int32_t* vnets, const int32_t* c,
                         const int32_t* w, int32_t k, int64_t lmax, int32_t* part,
                         uint8_t* eligible, uint8_t* moved, or_round_stats* st, int64_t* sgain);

/* One synchronous round; see lp_round_impl below. */
int or_lp_round(int32_t n, int32_t m, const int64_t* eptr, const int32_t* pins,
                const int64_t* vptr, const int32_t* vnets, const int32_t* c,
                const int32_t* w, int32_t k, int64_t lmax, int32_t* part,
                uint8_t* eligible, uint8_t* moved, or_round_stats* st) {
  return lp_round_impl(n, m, eptr, pins, vptr, vnets, c, w, k, lmax, part, eligible, moved, st,
                       NULL);
}

/* The same round, also reporting the select gain of every approved move
 * (sgain[u], n entries; other entries untouched). */
static int or_lp_round_gains(int32_t n, int32_t m, const int64_t* eptr, const int32_t* pins,
                             const int64_t* vptr, const int32_t* vnets, const int32_t* c,
                             const int32_t* w, int32_t k, int64_t lmax, int32_t* part,
                             uint8_t* eligible, uint8_t* moved, or_round_stats* st,
                             int64_t* sgain) {
  return lp_round_impl(n, m, eptr, pins, vptr, vnets, c, w, k, lmax, part, eligible, moved, st,
                       sgain);
}

static int lp_round_impl(int32_t n, int32_t m, const int64_t* eptr, const int32_t* pins,
                         const int64_t* vptr, const int32_t* vnets, const int32_t* c,
                         const int32_t* w, int32_t k, int64_t lmax, int32_t* part,
                         uint8_t* eligible, uint8_t* moved, or_round_stats* st, int64_t* sgain) {
  int32_t* phi = (int32_t*)malloc(sizeof(int32_t) * (size_t)m * (size_t)k);
  int32_t* lambda = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  int64_t* W = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  int64_t* conn = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  int32_t* target = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  or_cand* cand = (or_cand*)malloc(sizeof(or_cand) * (size_t)n);
  uint8_t* touched = (uint8_t*)malloc((size_t)m);
  if (!phi || !lambda || !W || !conn || !target || !cand || !touched) return OR_ERR_INVALID;
  memset(st, 0, sizeof(*st));

  /* round-start state S_r */
  or_pin_counts(m, eptr, pins, part, k, phi);
  int32_t wk = (k + 31) / 32;
  uint32_t* conn_bits = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)m * (size_t)wk);
  or_connectivity(m, k, phi, lambda, conn_bits);
  free(conn_bits);
  or_block_weights(n, c, part, k, W);
  int64_t km1_before = or_km1(m, w, lambda);

  /* steps 1-3: select */
  int64_t ncand = 0;
  for (int32_t u = 0; u < n; ++u) {
    target[u] = -1;
    if (!eligible[u]) continue;
    st->eligible += 1;
    int boundary = 0;
    for (int64_t j = vptr[u]; j < vptr[u + 1]; ++j)
      if (lambda[vnets[j]] > 1) boundary = 1;
    if (!boundary) continue;
    st->boundary += 1;
    st->active_pins += vptr[u + 1] - vptr[u];

    int32_t a = part[u];
    /* b(u) and, for every block, the weight of incident nets that already
     * touch that block: p_i(u) = w(I(u)) - conn_i.  A block i is a
     * neighbouring block iff some incident net has a pin in it. */
    int64_t b = 0, wsum = 0;
    for (int32_t i = 0; i < k; ++i) conn[i] = 0;
    for (int64_t j = vptr[u]; j < vptr[u + 1]; ++j) {
      int32_t e = vnets[j];
      wsum += ww(w, e);
      if (phi[(int64_t)e * k + a] == 1) b += ww(w, e);
      for (int32_t i = 0; i < k; ++i)
        if (phi[(int64_t)e * k + i] > 0) conn[i] += ww(w, e);
    }
    int32_t best = -1;
    int64_t best_gain = 0;
    for (int32_t i = 0; i < k; ++i) {
      if (i == a || conn[i] == 0) continue;         /* not a neighbouring block */
      if (W[i] + cw(c, u) > lmax) continue;         /* infeasible               */
      int64_t g = b - (wsum - conn[i]);             /* b(u) - p_i(u)            */
      if (best < 0 || g > best_gain || (g == best_gain && W[i] < W[best])) {
        best = i;                                   /* ties on (g, W): lower i  */
        best_gain = g;                              /* wins since i ascends     */
      }
    }
    if (best < 0) continue;
    int is_cand = best_gain > 0 || (best_gain == 0 && W[best] + cw(c, u) < W[a]);
    if (!is_cand) continue;
    cand[ncand].gain = best_gain;
    cand[ncand].u = u;
    cand[ncand].t = best;
    ncand += 1;
  }
  st->candidates = ncand;

  /* step 4: approval per target block, in (gain desc, id asc) order */
  qsort(cand, (size_t)ncand, sizeof(or_cand), cmp_cand);
  int64_t i0 = 0;
  while (i0 < ncand) {
    int32_t t = cand[i0].t;
    int64_t i1 = i0;
    while (i1 < ncand && cand[i1].t == t) ++i1;
    int64_t load = W[t];
    for (int64_t i = i0; i < i1; ++i) {
      if (load + cw(c, cand[i].u) > lmax) break;   /* longest feasible prefix */
      load += cw(c, cand[i].u);
      target[cand[i].u] = t;
      if (sgain) sgain[cand[i].u] = cand[i].gain;
    }
    i0 = i1;
  }

  /* step 5: apply all approved moves at once */
  memset(touched, 0, (size_t)m);
  for (int32_t u = 0; u < n; ++u) {
    moved[u] = 0;
  }
  for (int32_t u = 0; u < n; ++u) {
    if (target[u] < 0) continue;
    part[u] = target[u];
    moved[u] = 1;
    st->approved += 1;
    st->moved_pins += vptr[u + 1] - vptr[u];
    for (int64_t j = vptr[u]; j < vptr[u + 1]; ++j) touched[vnets[j]] = 1;
  }
  memset(eligible, 0, (size_t)n);
  for (int32_t e = 0; e < m; ++e) {
    if (!touched[e]) continue;
    st->touched_nets += 1;
    st->touched_pins += eptr[e + 1] - eptr[e];
    for (int64_t p = eptr[e]; p < eptr[e + 1]; ++p) eligible[pins[p]] = 1;
  }

  /* new state, recomputed from scratch */
  or_pin_counts(m, eptr, pins, part, k, phi);
  conn_bits = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)m * (size_t)wk);
  or_connectivity(m, k, phi, lambda, conn_bits);
  free(conn_bits);
  or_block_weights(n, c, part, k, W);
  st->km1_after = or_km1(m, w, lambda);
  st->km1_delta = km1_before - st->km1_after;
  st->max_block_weight = W[0];
  for (int32_t i = 1; i < k; ++i) if (W[i] > st->max_block_weight) st->max_block_weight = W[i];

  free(phi); free(lambda); free(W); free(conn); free(target); free(cand); free(touched);
  return OR_OK;
}

/* Refinement driver: R synchronous rounds from the given partition, every
 * vertex eligible in round 1 (section "Label Propagation": in the first round
 * every boundary vertex may move; afterwards the movers and their neighbours).
 * stats holds R records; rounds after convergence are recorded as empty.
 * Returns the final km1 through *km1_out. */
int or_refine(int32_t n, int32_t m, const int64_t* eptr, const int32_t* pins,
              const int32_t* c, const int32_t* w, int32_t k, int64_t lmax,
              int32_t rounds, int32_t* part, or_round_stats* stats, int64_t* km1_out) {
  int64_t* vptr = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int64_t P = eptr[m];
  int32_t* vnets = (int32_t*)malloc(sizeof(int32_t) * (size_t)P);
  uint8_t* eligible = (uint8_t*)malloc((size_t)n);
  uint8_t* moved = (uint8_t*)malloc((size_t)n);
  if (!vptr || !vnets || !eligible || !moved) return OR_ERR_INVALID;
  or_incidence(n, m, eptr, pins, vptr, vnets);
  memset(eligible, 1, (size_t)n);
  int rc = OR_OK;
  for (int32_t r = 0; r < rounds && rc == OR_OK; ++r)
    rc = or_lp_round(n, m, eptr, pins, vptr, vnets, c, w, k, lmax, part, eligible,
                     moved, &stats[r]);
  if (rc == OR_OK) {
    int32_t* phi = (int32_t*)malloc(sizeof(int32_t) * (size_t)m * (size_t)k);
    int32_t* lambda = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    uint32_t* conn_bits =
        (uint32_t*)malloc(sizeof(uint32_t) * (size_t)m * (size_t)((k + 31) / 32));
    or_pin_counts(m, eptr, pins, part, k, phi);
    or_connectivity(m, k, phi, lambda, conn_bits);
    *km1_out = or_km1(m, w, lambda);
    free(phi); free(lambda); free(conn_bits);
  }
  free(vptr); free(vnets); free(eligible); free(moved);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Move sequences (section "Parallel Gain Calculation", subsection "Parallel */
/* Gain Recalculation"; section "Direct k-way FM": best prefix).             */
/* ------------------------------------------------------------------------ */

/* Exact gain of every move of a sequence, as if the moves were performed one
 * after the other in the given order: move j takes vertex mu[j] from its
 * current block a to block mt[j] = b, and its gain is
 *   w({e in I(u) : Phi(e, a) = 1}) - w({e in I(u) : Phi(e, b) = 0})
 * on the pin counts left by moves 0..j-1 (the km1 decrease of that move).
 * Done literally: Phi is built from `part` and updated move by move.  part is
 * the partition before the sequence and is not changed.  Returns
 * OR_ERR_INVALID if a vertex moves twice, a target lies outside [0,k) or a
 * move targets the block its vertex is in. */
int or_move_gains(int32_t n, int32_t m, const int64_t* eptr, const int32_t* pins,
                  const int64_t* vptr, const int32_t* vnets, const int32_t* w, int32_t k,
                  const int32_t* part, int32_t t, const int32_t* mu, const int32_t* mt,
                  int64_t* gains) {
  int32_t* phi = (int32_t*)malloc(sizeof(int32_t) * (size_t)m * (size_t)k);
  int32_t* cur = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  uint8_t* seen = (uint8_t*)calloc((size_t)n, 1);
  if (!phi || !cur || !seen) return OR_ERR_INVALID;
  or_pin_counts(m, eptr, pins, part, k, phi);
  memcpy(cur, part, sizeof(int32_t) * (size_t)n);
  int rc = OR_OK;
  for (int32_t j = 0; j < t && rc == OR_OK; ++j) {
    const int32_t u = mu[j], b = mt[j];
    if (u < 0 || u >= n || seen[u] || b < 0 || b >= k || cur[u] == b) {
      rc = OR_ERR_INVALID;
      break;
    }
    seen[u] = 1;
    const int32_t a = cur[u];
    int64_t g = 0;
    for (int64_t q = vptr[u]; q < vptr[u + 1]; ++q) {
      const int32_t e = vnets[q];
      if (phi[(int64_t)e * k + a] == 1) g += ww(w, e);
      if (phi[(int64_t)e * k + b] == 0) g -= ww(w, e);
    }
    gains[j] = g;
    for (int64_t q = vptr[u]; q < vptr[u + 1]; ++q) {
      const int32_t e = vnets[q];
      phi[(int64_t)e * k + a] -= 1;
      phi[(int64_t)e * k + b] += 1;
    }
    cur[u] = b;
  }
  free(phi); free(cur); free(seen);
  return rc;
}

/* Best prefix of a move sequence: the length p in [0, t] with the largest
 * total gain gains[0] + ... + gains[p-1] among the prefixes after which every
 * block weight is at most lmax; the empty prefix always qualifies; ties go to
 * the longer prefix.  Block weights are followed move by move from `part`. */
void or_best_prefix(int32_t n, const int32_t* c, int32_t k, int64_t lmax, const int32_t* part,
                    int32_t t, const int32_t* mu, const int32_t* mt, const int64_t* gains,
                    int32_t* best_len, int64_t* best_gain) {
  int64_t* W = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  int32_t* cur = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  or_block_weights(n, c, part, k, W);
  memcpy(cur, part, sizeof(int32_t) * (size_t)n);
  int64_t over = 0, total = 0;
  for (int32_t i = 0; i < k; ++i) over += W[i] > lmax;
  *best_len = 0;
  *best_gain = 0;
  for (int32_t j = 0; j < t; ++j) {
    const int32_t u = mu[j], a = cur[u], b = mt[j];
    over -= (W[a] > lmax) + (W[b] > lmax);
    W[a] -= cw(c, u);
    W[b] += cw(c, u);
    over += (W[a] > lmax) + (W[b] > lmax);
    cur[u] = b;
    total += gains[j];
    if (over == 0 && total >= *best_gain) {
      *best_len = j + 1;
      *best_gain = total;
    }
  }
  free(W); free(cur);
}

/* One monotone label-propagation round: candidates and approval exactly as in
 * or_lp_round; the approved moves, ordered by (select gain desc, vertex id
 * asc), get their exact gains in that order (or_move_gains) and only the
 * prefix with the largest total gain is applied (or_best_prefix, ties to the
 * longer prefix; every prefix of approved moves respects L_max, because the
 * approval already budgets each target block for all of its moves and moves
 * out of a block only lower its weight).  km1 never increases.  The stats are
 * those of or_lp_round with `approved` = the prefix length; the approved set
 * before the cut is returned in *n_approved when non-NULL. */
int or_lp_round_exact(int32_t n, int32_t m, const int64_t* eptr, const int32_t* pins,
                      const int64_t* vptr, const int32_t* vnets, const int32_t* c,
                      const int32_t* w, int32_t k, int64_t lmax, int32_t* part,
                      uint8_t* eligible, uint8_t* moved, or_round_stats* st,
                      int64_t* n_approved) {
  /* a plain round on copies gives the approved set and its select gains */
  int32_t* part2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  uint8_t* elig2 = (uint8_t*)malloc((size_t)n);
  int64_t* sgain = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  or_cand* seq = (or_cand*)malloc(sizeof(or_cand) * (size_t)n);
  int32_t* mu = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* mt = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int64_t* gains = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  uint8_t* touched = (uint8_t*)malloc((size_t)m);
  if (!part2 || !elig2 || !sgain || !seq || !mu || !mt || !gains || !touched)
    return OR_ERR_INVALID;
  memcpy(part2, part, sizeof(int32_t) * (size_t)n);
  memcpy(elig2, eligible, (size_t)n);
  or_round_stats plain;
  int rc = or_lp_round_gains(n, m, eptr, pins, vptr, vnets, c, w, k, lmax, part2, elig2, moved,
                             &plain, sgain);
  if (rc != OR_OK) return rc;
  /* the approved moves in (gain desc, id asc) order */
  int64_t t = 0;
  for (int32_t u = 0; u < n; ++u) {
    if (!moved[u]) continue;
    seq[t].gain = sgain[u];
    seq[t].u = u;
    seq[t].t = part2[u];
    t += 1;
  }
  qsort(seq, (size_t)t, sizeof(or_cand), cmp_gain_id);
  for (int64_t j = 0; j < t; ++j) {
    mu[j] = seq[j].u;
    mt[j] = seq[j].t;
  }
  rc = or_move_gains(n, m, eptr, pins, vptr, vnets, w, k, part, (int32_t)t, mu, mt, gains);
  if (rc != OR_OK) return rc;
  int32_t p = 0;
  int64_t best = 0;
  /* lmax = INT64_MAX: the prefixes are feasible by construction (see above) */
  or_best_prefix(n, c, k, INT64_MAX, part, (int32_t)t, mu, mt, gains, &p, &best);
  if (n_approved) *n_approved = t;

  /* apply the prefix, then the round record as in or_lp_round */
  *st = plain;
  st->approved = p;
  st->moved_pins = 0;
  st->touched_nets = 0;
  st->touched_pins = 0;
  int32_t* phi = (int32_t*)malloc(sizeof(int32_t) * (size_t)m * (size_t)k);
  int32_t* lambda = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  uint32_t* bits = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)m * (size_t)((k + 31) / 32));
  int64_t* W = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  or_pin_counts(m, eptr, pins, part, k, phi);
  or_connectivity(m, k, phi, lambda, bits);
  const int64_t km1_before = or_km1(m, w, lambda);
  memset(moved, 0, (size_t)n);
  memset(touched, 0, (size_t)m);
  for (int32_t j = 0; j < p; ++j) {
    const int32_t u = mu[j];
    part[u] = mt[j];
    moved[u] = 1;
    st->moved_pins += vptr[u + 1] - vptr[u];
    for (int64_t q = vptr[u]; q < vptr[u + 1]; ++q) touched[vnets[q]] = 1;
  }
  memset(eligible, 0, (size_t)n);
  for (int32_t e = 0; e < m; ++e) {
    if (!touched[e]) continue;
    st->touched_nets += 1;
    st->touched_pins += eptr[e + 1] - eptr[e];
    for (int64_t q = eptr[e]; q < eptr[e + 1]; ++q) eligible[pins[q]] = 1;
  }
  or_pin_counts(m, eptr, pins, part, k, phi);
  or_connectivity(m, k, phi, lambda, bits);
  or_block_weights(n, c, part, k, W);
  st->km1_after = or_km1(m, w, lambda);
  st->km1_delta = km1_before - st->km1_after;
  st->max_block_weight = W[0];
  for (int32_t i = 1; i < k; ++i) if (W[i] > st->max_block_weight) st->max_block_weight = W[i];
  free(part2); free(elig2); free(sgain); free(seq); free(mu); free(mt); free(gains);
  free(touched); free(phi); free(lambda); free(bits); free(W);
  return OR_OK;
}

/* Refinement driver of the monotone variant: as or_refine with
 * or_lp_round_exact in place of or_lp_round. */
int or_refine_exact(int32_t n, int32_t m, const int64_t* eptr, const int32_t* pins,
                    const int32_t* c, const int32_t* w, int32_t k, int64_t lmax,
                    int32_t rounds, int32_t* part, or_round_stats* stats, int64_t* km1_out) {
  int64_t* vptr = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int64_t P = eptr[m];
  int32_t* vnets = (int32_t*)malloc(sizeof(int32_t) * (size_t)P);
  uint8_t* eligible = (uint8_t*)malloc((size_t)n);
  uint8_t* moved = (uint8_t*)malloc((size_t)n);
  if (!vptr || !vnets || !eligible || !moved) return OR_ERR_INVALID;
  or_incidence(n, m, eptr, pins, vptr, vnets);
  memset(eligible, 1, (size_t)n);
  int rc = OR_OK;
  for (int32_t r = 0; r < rounds && rc == OR_OK; ++r)
    rc = or_lp_round_exact(n, m, eptr, pins, vptr, vnets, c, w, k, lmax, part, eligible, moved,
                           &stats[r], NULL);
  if (rc == OR_OK) {
    int32_t* phi = (int32_t*)malloc(sizeof(int32_t) * (size_t)m * (size_t)k);
    int32_t* lambda = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
    uint32_t* bits = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)m * (size_t)((k + 31) / 32));
    or_pin_counts(m, eptr, pins, part, k, phi);
    or_connectivity(m, k, phi, lambda, bits);
    *km1_out = or_km1(m, w, lambda);
    free(phi); free(lambda); free(bits);
  }
  free(vptr); free(vnets); free(eligible); free(moved);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Rebalancing (section "Rebalancing"), one synchronous deterministic round. */
/* The paper moves vertices out of overloaded blocks, non-negative gains     */
/* first (at once) and then the least-loss moves from priority queues, while */
/* the block is still overloaded.  Read for a synchronous round:             */
/*  1. overloaded blocks O = {a : c(V_a) > L_max}; every vertex u of a block */
/*     in O is considered;                                                   */
/*  2. its target is the best block i != Pi(u) with c(V_i) + c(u) <= L_max  */
/*     -- any block, not only neighbouring ones -- by (g_i(u) desc, c(V_i)  */
/*     asc, i asc), g_i(u) = b(u) - p_i(u) of any sign; none: no candidate;  */
/*  3. per source block a, candidates in (gain desc, id asc) order: the      */
/*     shortest prefix whose weight reaches the excess c(V_a) - L_max is     */
/*     proposed (all of them if the total falls short) -- gain order puts    */
/*     the non-negative moves first and then the smallest losses;            */
/*  4. per target block t, proposed moves in (gain desc, id asc) order: the  */
/*     longest prefix with c(V_t) + prefix weight <= L_max is approved;      */
/*  5. approved moves are applied at once; pins of nets holding a moved      */
/*     vertex become eligible (for label propagation afterwards).            */
/* All decisions read the round-start state.  The record: eligible = vertices*/
/* considered, boundary = moves proposed, candidates = vertices with a       */
/* target, approved = moves applied, active_pins = sum of d(u) over the      */
/* considered vertices; the other fields as in a label-propagation round.    */
/* A balanced partition is left unchanged (an empty record).                  */
/* ------------------------------------------------------------------------ */

typedef struct { int64_t gain; int32_t u; int32_t a; int32_t t; int32_t c; } or_rb_cand;

static int cmp_rb_source(const void* x, const void* y) {
  const or_rb_cand* a = (const or_rb_cand*)x;
  const or_rb_cand* b = (const or_rb_cand*)y;
  if (a->a != b->a) return a->a < b->a ? -1 : 1;
  if (a->gain != b->gain) return a->gain > b->gain ? -1 : 1;
  return (a->u > b->u) - (a->u < b->u);
}

static int cmp_rb_target(const void* x, const void* y) {
  const or_rb_cand* a = (const or_rb_cand*)x;
  const or_rb_cand* b = (const or_rb_cand*)y;
  if (a->t != b->t) return a->t < b->t ? -1 : 1;
  if (a->gain != b->gain) return a->gain > b->gain ? -1 : 1;
  return (a->u > b->u) - (a->u < b->u);
}

int or_rebalance_round(int32_t n, int32_t m, const int64_t* eptr, const int32_t* pins,
                       const int64_t* vptr, const int32_t* vnets, const int32_t* c,
                       const int32_t* w, int32_t k, int64_t lmax, int32_t* part,
                       uint8_t* eligible, uint8_t* moved, or_round_stats* st) {
  int32_t* phi = (int32_t*)malloc(sizeof(int32_t) * (size_t)m * (size_t)k);
  int32_t* lambda = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  uint32_t* bits = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)m * (size_t)((k + 31) / 32));
  int64_t* W = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  int64_t* acc = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  int64_t* gains = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
  or_rb_cand* cand = (or_rb_cand*)malloc(sizeof(or_rb_cand) * (size_t)n + 1);
  uint8_t* touched = (uint8_t*)malloc((size_t)m);
  if (!phi || !lambda || !bits || !W || !acc || !gains || !cand || !touched) return OR_ERR_INVALID;
  memset(st, 0, sizeof(*st));
  or_pin_counts(m, eptr, pins, part, k, phi);
  or_connectivity(m, k, phi, lambda, bits);
  const int64_t km1_before = or_km1(m, w, lambda);
  or_block_weights(n, c, part, k, W);

  /* steps 1-2: candidates of the overloaded blocks */
  int32_t nc = 0;
  for (int32_t u = 0; u < n; ++u) {
    moved[u] = 0;
    const int32_t a = part[u];
    if (W[a] <= lmax) continue;
    st->eligible += 1;
    st->active_pins += vptr[u + 1] - vptr[u];
    /* g_i(u) = b(u) - p_i(u) for every block, from the pin counts */
    int64_t b = 0;
    for (int32_t i = 0; i < k; ++i) gains[i] = 0;
    for (int64_t j = vptr[u]; j < vptr[u + 1]; ++j) {
      const int32_t e = vnets[j];
      if (phi[(int64_t)e * k + a] == 1) b += ww(w, e);
      for (int32_t i = 0; i < k; ++i)
        if (phi[(int64_t)e * k + i] == 0) gains[i] -= ww(w, e);
    }
    int32_t t = -1;
    for (int32_t i = 0; i < k; ++i) {
      if (i == a || W[i] + cw(c, u) > lmax) continue;
      const int64_t g = b + gains[i];
      if (t < 0 || g > b + gains[t] || (g == b + gains[t] && (W[i] < W[t] ||
                                                              (W[i] == W[t] && i < t))))
        t = i;
    }
    if (t < 0) continue;
    cand[nc].gain = b + gains[t];
    cand[nc].u = u;
    cand[nc].a = a;
    cand[nc].t = t;
    cand[nc].c = (int32_t)cw(c, u);
    ++nc;
  }
  st->candidates = nc;

  /* step 3: shortest prefix per source reaching its excess */
  qsort(cand, (size_t)nc, sizeof(or_rb_cand), cmp_rb_source);
  for (int32_t i = 0; i < k; ++i) acc[i] = 0;
  int32_t np = 0;
  for (int32_t j = 0; j < nc; ++j) {
    const int32_t a = cand[j].a;
    if (acc[a] < W[a] - lmax) {
      acc[a] += cand[j].c;
      cand[np++] = cand[j];
    }
  }
  st->boundary = np;

  /* step 4: longest prefix per target that fits */
  qsort(cand, (size_t)np, sizeof(or_rb_cand), cmp_rb_target);
  for (int32_t i = 0; i < k; ++i) acc[i] = 0;
  int32_t closed_t = -1;
  memset(touched, 0, (size_t)m);
  for (int32_t j = 0; j < np; ++j) {
    const int32_t t = cand[j].t, u = cand[j].u;
    if (t == closed_t) continue;
    if (W[t] + acc[t] + cand[j].c > lmax) {
      closed_t = t;            /* the prefix of this target ends here */
      continue;
    }
    acc[t] += cand[j].c;
    /* step 5 (applied below, after every decision is taken) */
    moved[u] = 1;
    st->approved += 1;
    st->moved_pins += vptr[u + 1] - vptr[u];
  }
  for (int32_t j = 0; j < np; ++j)
    if (moved[cand[j].u]) part[cand[j].u] = cand[j].t;
  for (int32_t u = 0; u < n; ++u)
    if (moved[u])
      for (int64_t j = vptr[u]; j < vptr[u + 1]; ++j) touched[vnets[j]] = 1;
  for (int32_t e = 0; e < m; ++e) {
    if (!touched[e]) continue;
    st->touched_nets += 1;
    st->touched_pins += eptr[e + 1] - eptr[e];
    for (int64_t p = eptr[e]; p < eptr[e + 1]; ++p) eligible[pins[p]] = 1;
  }
  or_pin_counts(m, eptr, pins, part, k, phi);
  or_connectivity(m, k, phi, lambda, bits);
  or_block_weights(n, c, part, k, W);
  st->km1_after = or_km1(m, w, lambda);
  st->km1_delta = km1_before - st->km1_after;
  st->max_block_weight = W[0];
  for (int32_t i = 1; i < k; ++i) if (W[i] > st->max_block_weight) st->max_block_weight = W[i];
  free(phi); free(lambda); free(bits); free(W); free(acc); free(gains); free(cand); free(touched);
  return OR_OK;
}

/* `rounds` rebalancing rounds (every one recorded; once balanced, or once a */
/* round moves nothing, the later rounds are empty).  eligible is updated as */
/* each round says; *km1_out = km1 at the end.                               */
int or_rebalance(int32_t n, int32_t m, const int64_t* eptr, const int32_t* pins,
                 const int32_t* c, const int32_t* w, int32_t k, int64_t lmax, int32_t rounds,
                 int32_t* part, uint8_t* eligible, or_round_stats* stats, int64_t* km1_out) {
  int64_t* vptr = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t* vnets = (int32_t*)malloc(sizeof(int32_t) * (size_t)eptr[m] + 1);
  uint8_t* moved = (uint8_t*)malloc((size_t)n);
  int32_t* phi = (int32_t*)malloc(sizeof(int32_t) * (size_t)m * (size_t)k);
  int32_t* lambda = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  uint32_t* bits = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)m * (size_t)((k + 31) / 32));
  if (!vptr || !vnets || !moved || !phi || !lambda || !bits) return OR_ERR_INVALID;
  or_incidence(n, m, eptr, pins, vptr, vnets);
  int rc = OR_OK;
  for (int32_t r = 0; r < rounds && rc == OR_OK; ++r)
    rc = or_rebalance_round(n, m, eptr, pins, vptr, vnets, c, w, k, lmax, part, eligible, moved,
                            &stats[r]);
  or_pin_counts(m, eptr, pins, part, k, phi);
  or_connectivity(m, k, phi, lambda, bits);
  *km1_out = or_km1(m, w, lambda);
  free(vptr); free(vnets); free(moved); free(phi); free(lambda); free(bits);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Contraction (section "Coarsening", subsection "Contraction") of a vertex  */
/* clustering cluster[v] in [0, n):                                          */
/*  1. cluster ids are renumbered to 0..n'-1 in increasing id order (the    */
/*     rank of the id among the used ones): map[v];                          */
/*  2. c'(x) = sum of c(v) over map[v] = x;                                  */
/*  3. every net's pins are mapped and duplicates removed; the pins of a     */
/*     coarse net are listed in increasing order;                            */
/*  4. nets left with a single pin are dropped;                              */
/*  5. nets with the same pin set are one net whose weight is the sum; it    */
/*     keeps the place of the lowest original net id among them;            */
/*  6. coarse nets are numbered in increasing order of those ids.            */
/* Written from the definition: identical nets are found by sorting the     */
/* nets by (size, pins) and comparing neighbours; no fingerprints.           */
/* Outputs (capacity n, n, m+1, P, m): map, cvwgt, ceptr, cpins, cewgt;      */
/* sizes[0..2] = n', m', P'.  Returns OR_ERR_INVALID for a cluster id        */
/* outside [0, n) and OR_ERR_UNSUPPORTED when a cluster weighs >= 2^31.      */
/* ------------------------------------------------------------------------ */

typedef struct { const int32_t* pins; int64_t size; int32_t id; } or_net_ref;

static int cmp_net_ref(const void* x, const void* y) {
  const or_net_ref* a = (const or_net_ref*)x;
  const or_net_ref* b = (const or_net_ref*)y;
  if (a->size != b->size) return a->size < b->size ? -1 : 1;
  for (int64_t i = 0; i < a->size; ++i)
    if (a->pins[i] != b->pins[i]) return a->pins[i] < b->pins[i] ? -1 : 1;
  return (a->id > b->id) - (a->id < b->id);
}

int or_contract(int32_t n, int32_t m, const int64_t* eptr, const int32_t* pins,
                const int32_t* c, const int32_t* w, const int32_t* cluster, int32_t* map,
                int32_t* cvwgt, int64_t* ceptr, int32_t* cpins, int32_t* cewgt,
                int64_t* sizes) {
  if (n < 1 || m < 0) return OR_ERR_INVALID;
  const size_t nn = (size_t)(uint32_t)n;
  for (int32_t v = 0; v < n; ++v)
    if (cluster[v] < 0 || cluster[v] >= n) return OR_ERR_INVALID;
  /* 1. renumbering */
  int32_t* rank = (int32_t*)calloc(nn, sizeof(int32_t));
  uint8_t* used = (uint8_t*)calloc(nn, 1);
  for (int32_t v = 0; v < n; ++v) used[cluster[v]] = 1;
  int32_t nc = 0;
  for (int32_t i = 0; i < n; ++i) {
    rank[i] = nc;
    nc += used[i];
  }
  for (int32_t v = 0; v < n; ++v) map[v] = rank[cluster[v]];
  /* 2. weights */
  int64_t* cw64 = (int64_t*)calloc(nn, sizeof(int64_t));
  for (int32_t v = 0; v < n; ++v) cw64[map[v]] += cw(c, v);
  int rc = OR_OK;
  for (int32_t x = 0; x < nc; ++x) {
    if (cw64[x] > 0x7fffffffLL) rc = OR_ERR_UNSUPPORTED;
    cvwgt[x] = (int32_t)cw64[x];
  }
  /* 3-4. mapped, sorted, deduplicated pins; single-pin nets dropped */
  const int64_t P = eptr[m];
  int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(P + 1));
  int64_t* tsize = (int64_t*)calloc((size_t)m + 1, sizeof(int64_t));
  for (int32_t e = 0; e < m; ++e) {
    int32_t* t = tmp + eptr[e];
    const int64_t s = eptr[e + 1] - eptr[e];
    for (int64_t i = 0; i < s; ++i) t[i] = map[pins[eptr[e] + i]];
    qsort(t, (size_t)s, sizeof(int32_t), cmp_i32);
    int64_t d = 0;
    for (int64_t i = 0; i < s; ++i)
      if (i == 0 || t[i] != t[i - 1]) t[d++] = t[i];
    tsize[e] = d;
  }
  /* 5. identical nets: sort by (size, pins, id), equal neighbours merge */
  or_net_ref* ref = (or_net_ref*)malloc(sizeof(or_net_ref) * ((size_t)m + 1));
  int32_t* rep = (int32_t*)malloc(sizeof(int32_t) * ((size_t)m + 1));
  int64_t* wsum = (int64_t*)calloc((size_t)m + 1, sizeof(int64_t));
  int32_t nr = 0;
  for (int32_t e = 0; e < m; ++e) {
    rep[e] = -1;
    if (tsize[e] < 2) continue;
    ref[nr].pins = tmp + eptr[e];
    ref[nr].size = tsize[e];
    ref[nr].id = e;
    ++nr;
  }
  qsort(ref, (size_t)nr, sizeof(or_net_ref), cmp_net_ref);
  for (int32_t j = 0; j < nr; ++j) {
    const int same = j > 0 && ref[j].size == ref[j - 1].size &&
                     memcmp(ref[j].pins, ref[j - 1].pins, sizeof(int32_t) * (size_t)ref[j].size) == 0;
    rep[ref[j].id] = same ? rep[ref[j - 1].id] : ref[j].id;   /* lowest id comes first */
    wsum[rep[ref[j].id]] += ww(w, ref[j].id);
  }
  /* 6. output in increasing representative id */
  int32_t mc = 0;
  int64_t pc = 0;
  ceptr[0] = 0;
  for (int32_t e = 0; e < m; ++e) {
    if (rep[e] != e) continue;
    for (int64_t i = 0; i < tsize[e]; ++i) cpins[pc++] = tmp[eptr[e] + i];
    cewgt[mc] = (int32_t)wsum[e];
    ceptr[++mc] = pc;
  }
  sizes[0] = nc;
  sizes[1] = mc;
  sizes[2] = pc;
  free(rank); free(used); free(cw64); free(tmp); free(tsize); free(ref); free(rep); free(wsum);
  return rc;
}
