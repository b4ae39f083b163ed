/*
 * bcd_oracle.c -- plain, slow, obviously-correct CPU oracle for the
 * betweenness of one vertex r in a directed graph, restricted to the
 * sources that can reach r (Chehreghani, Bifet and Abdessalem, "Exact and
 * approximate algorithms for computing betweenness centrality in directed
 * graphs").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * bench's CPU-baseline leg load this file.  It shares no code, header,
 * table or helper with the GPU library; the two meet only through the
 * seeded inputs they are both given.
 *
 * Paper references are by section / equation / algorithm / proposition:
 *   Eq.(1)  BC(v) = sum over s != v != t of sigma_st(v) / sigma_st
 *   Eq.(2)  dependency delta_s.(v) = sum_t sigma_st(v)/sigma_st
 *   Eq.(3)  BC(v) = sum_{s != v} delta_s.(v)
 *   Eq.(4)  delta_s.(v) = sum_{w : v in P_s(w)} sigma_sv/sigma_sw (1 + delta_s.(w))
 *   Def.1 / Prop.1 / Eq.(5)  BC(r) = sum over v in RV(r) of delta_v.(r),
 *                            and 0 when r has out-degree 0
 *   Def.2, Def.3, Prop.2     RV(r) = vertices met by a BFS from r on the
 *                            reverse graph (weights ignored), minus r
 *   Alg.1 (E-BCD), the set variant of Section 4.2, Alg.2 (A-BCD)
 *   Eq.(8)  T >= ln(2/delta) K^2 |RV(r)|^2 / (2 eps^2)
 *
 * Types (the paper fixes none): distances uint64, sigma uint64 with every
 * addition checked for wrap-around, dependencies accumulated in long double
 * and rounded to double once per source.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
  OR_OK = 0,
  OR_INVALID = 1,
  OR_BAD_GRAPH = 2,
  OR_OVERFLOW = 3,
  OR_NOMEM = 4,
  OR_TOO_SMALL = 6
};

#define OR_INF UINT64_MAX

typedef struct {
  int64_t n, m;
  const int64_t *rp;
  const int32_t *col;
  const uint32_t *w; /* NULL: every arc has length 1 */
} og;

/* per-source traversal counters: reached vertices, arcs leaving them,
   shortest-path-DAG arcs */
typedef struct {
  uint64_t n_s, m_s, a_s;
} oc;

/* ------------------------------------------------------------------ graph */

int oracle_check_graph(int64_t n, int64_t m, const int64_t *rp, const int32_t *col,
                       const uint32_t *w) {
  if (n <= 0 || n >= ((int64_t)1 << 31) || m < 0 || !rp || (m > 0 && !col)) return OR_INVALID;
  if (rp[0] != 0 || rp[n] != m) return OR_BAD_GRAPH;
  for (int64_t v = 0; v < n; ++v) {
    if (rp[v + 1] < rp[v]) return OR_BAD_GRAPH;
    for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
      if (col[e] < 0 || col[e] >= n || col[e] == v) return OR_BAD_GRAPH;
      if (e > rp[v] && col[e] <= col[e - 1]) return OR_BAD_GRAPH;
      if (w && w[e] == 0) return OR_BAD_GRAPH;
    }
  }
  return OR_OK;
}

/* ---------------------------------------------------- RV(r): Def.3, Prop.2
 * Build the reverse graph R(G) (Def.2), ignore weights, breadth-first search
 * from r, keep every vertex met except r.  Output ascending. */
int oracle_rv(int64_t n, int64_t m, const int64_t *rp, const int32_t *col, int32_t r,
              int32_t *out, int64_t cap, int64_t *count) {
  if (r < 0 || r >= n || !count) return OR_INVALID;
  int64_t *irp = calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *icol = malloc((size_t)(m ? m : 1) * sizeof(int32_t));
  int64_t *fill = malloc((size_t)n * sizeof(int64_t));
  char *seen = calloc((size_t)n, 1);
  int32_t *queue = malloc((size_t)n * sizeof(int32_t));
  if (!irp || !icol || !fill || !seen || !queue) {
    free(irp); free(icol); free(fill); free(seen); free(queue);
    return OR_NOMEM;
  }
  /* reverse graph: arc (u,v) of G becomes (v,u) */
  for (int64_t e = 0; e < m; ++e) irp[col[e] + 1]++;
  for (int64_t v = 0; v < n; ++v) irp[v + 1] += irp[v];
  for (int64_t v = 0; v < n; ++v) fill[v] = irp[v];
  for (int64_t u = 0; u < n; ++u)
    for (int64_t e = rp[u]; e < rp[u + 1]; ++e) icol[fill[col[e]]++] = (int32_t)u;
  /* BFS on R(G) from r */
  int64_t head = 0, tail = 0;
  queue[tail++] = r;
  seen[r] = 1;
  while (head < tail) {
    int32_t v = queue[head++];
    for (int64_t e = irp[v]; e < irp[v + 1]; ++e) {
      int32_t u = icol[e];
      if (!seen[u]) {
        seen[u] = 1;
        queue[tail++] = u;
      }
    }
  }
  int64_t k = 0;
  for (int64_t v = 0; v < n; ++v)
    if (seen[v] && v != r) k++;
  int st = OR_OK;
  if (out && k > cap) st = OR_TOO_SMALL;
  if (out && st == OR_OK) {
    int64_t j = 0;
    for (int64_t v = 0; v < n; ++v)
      if (seen[v] && v != r) out[j++] = (int32_t)v;
  }
  *count = k;
  free(irp); free(icol); free(fill); free(seen); free(queue);
  return st;
}

/* number of vertices reachable from r in G, r excluded (the bound K read
   for Prop.4) */
int oracle_fr_count(int64_t n, int64_t m, const int64_t *rp, const int32_t *col, int32_t r,
                    int64_t *count) {
  (void)m;
  if (r < 0 || r >= n || !count) return OR_INVALID;
  char *seen = calloc((size_t)n, 1);
  int32_t *queue = malloc((size_t)n * sizeof(int32_t));
  if (!seen || !queue) { free(seen); free(queue); return OR_NOMEM; }
  int64_t head = 0, tail = 0;
  queue[tail++] = r;
  seen[r] = 1;
  while (head < tail) {
    int32_t v = queue[head++];
    for (int64_t e = rp[v]; e < rp[v + 1]; ++e)
      if (!seen[col[e]]) { seen[col[e]] = 1; queue[tail++] = col[e]; }
  }
  *count = tail - 1;
  free(seen); free(queue);
  return OR_OK;
}

/* ------------------------------------------- one source: SPD + Eq.(4)
 * Forward: shortest-path distances d and path counts sigma from s (BFS when
 * unweighted, Dijkstra with a binary heap and lazy deletion when weighted),
 * recording the order in which vertices are settled.  Backward: walk the
 * settle order from last to first and evaluate Eq.(4) for each vertex v as
 * the sum over its SPD successors w (those with d(w) = d(v) + len(v,w)),
 * which are exactly the w with v in P_s(w). */

typedef struct {
  uint64_t *d;
  uint64_t *sigma;
  long double *delta;
  int32_t *order; /* settle order */
  /* heap for the weighted case */
  uint64_t *hk;
  int32_t *hv;
  int64_t hcap;
} oscratch;

static int scratch_init(oscratch *S, int64_t n, int64_t m) {
  memset(S, 0, sizeof(*S));
  S->d = malloc((size_t)n * sizeof(uint64_t));
  S->sigma = malloc((size_t)n * sizeof(uint64_t));
  S->delta = malloc((size_t)n * sizeof(long double));
  S->order = malloc((size_t)n * sizeof(int32_t));
  S->hcap = m + 2;
  S->hk = malloc((size_t)S->hcap * sizeof(uint64_t));
  S->hv = malloc((size_t)S->hcap * sizeof(int32_t));
  if (!S->d || !S->sigma || !S->delta || !S->order || !S->hk || !S->hv) return OR_NOMEM;
  return OR_OK;
}

static void scratch_free(oscratch *S) {
  free(S->d); free(S->sigma); free(S->delta); free(S->order); free(S->hk); free(S->hv);
}

static void heap_push(oscratch *S, int64_t *sz, uint64_t k, int32_t v) {
  int64_t i = (*sz)++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (S->hk[p] <= k) break;
    S->hk[i] = S->hk[p];
    S->hv[i] = S->hv[p];
    i = p;
  }
  S->hk[i] = k;
  S->hv[i] = v;
}

static void heap_pop(oscratch *S, int64_t *sz, uint64_t *k, int32_t *v) {
  *k = S->hk[0];
  *v = S->hv[0];
  int64_t last = --(*sz);
  uint64_t lk = S->hk[last];
  int32_t lv = S->hv[last];
  int64_t i = 0;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= last) break;
    if (c + 1 < last && S->hk[c + 1] < S->hk[c]) c++;
    if (S->hk[c] >= lk) break;
    S->hk[i] = S->hk[c];
    S->hv[i] = S->hv[c];
    i = c;
  }
  S->hk[i] = lk;
  S->hv[i] = lv;
}

/* checked sigma[w] += x; an already-wrapped addend is caught where it wrapped */
static inline void sigma_add(uint64_t *dst, uint64_t x, int *ovf) {
  uint64_t r = *dst + x;
  if (r < *dst) *ovf = 1;
  *dst = r;
}

/* Runs the forward pass from s.  Returns the number of settled vertices. */
static int64_t forward(const og *G, int32_t s, oscratch *S, int *ovf, oc *cnt) {
  const int64_t n = G->n;
  for (int64_t v = 0; v < n; ++v) { S->d[v] = OR_INF; S->sigma[v] = 0; }
  S->d[s] = 0;
  S->sigma[s] = 1;
  int64_t settled = 0;
  uint64_t msum = 0, asum = 0;
  if (!G->w) {
    /* BFS; order doubles as the FIFO queue */
    int64_t head = 0, tail = 0;
    S->order[tail++] = s;
    while (head < tail) {
      int32_t v = S->order[head++];
      msum += (uint64_t)(G->rp[v + 1] - G->rp[v]);
      for (int64_t e = G->rp[v]; e < G->rp[v + 1]; ++e) {
        int32_t w = G->col[e];
        if (S->d[w] == OR_INF) {
          S->d[w] = S->d[v] + 1;
          S->order[tail++] = w;
        }
        if (S->d[w] == S->d[v] + 1) {
          sigma_add(&S->sigma[w], S->sigma[v], ovf);
          asum++;
        }
      }
    }
    settled = tail;
  } else {
    /* Dijkstra; a vertex is settled when popped with its final distance.
       sigma[w] is reset on a strict improvement of d[w] and grows on a tie,
       so a tie at a tentative distance that is later beaten leaves no trace
       in the final sigma[w].  Its wrap-around must not either: wrap[w]
       records a wrapped add into sigma[w] at the current d[w] and is
       cleared with sigma[w].  Overflow is a FINAL count above 2^64 - 1, so
       the flag is raised from the wrap bits of the settled vertices once
       every distance is final.  (If some final sigma_s(v) exceeds 2^64 - 1,
       then at some vertex on the way the exact sum of its final
       predecessors' counts does, and that add wraps; the converse holds
       because a count that wrapped only feeds vertices whose own exact
       count is at least as large.) */
    char *done = calloc((size_t)n, 1);
    char *wrap = calloc((size_t)n, 1);
    int64_t hs = 0;
    heap_push(S, &hs, 0, s);
    while (hs > 0) {
      uint64_t dv;
      int32_t v;
      heap_pop(S, &hs, &dv, &v);
      if (done[v] || dv != S->d[v]) continue;
      done[v] = 1;
      S->order[settled++] = v;
      msum += (uint64_t)(G->rp[v + 1] - G->rp[v]);
      for (int64_t e = G->rp[v]; e < G->rp[v + 1]; ++e) {
        int32_t w = G->col[e];
        uint64_t nd = dv + G->w[e];
        if (nd < S->d[w]) {
          S->d[w] = nd;
          S->sigma[w] = S->sigma[v];
          wrap[w] = 0;
          heap_push(S, &hs, nd, w);
        } else if (nd == S->d[w]) {
          int c = 0;
          sigma_add(&S->sigma[w], S->sigma[v], &c);
          if (c) wrap[w] = 1;
        }
      }
    }
    for (int64_t i = 0; i < settled; ++i)
      if (wrap[S->order[i]]) *ovf = 1;
    free(done);
    free(wrap);
    /* SPD arcs, counted on the final distances */
    for (int64_t i = 0; i < settled; ++i) {
      int32_t v = S->order[i];
      for (int64_t e = G->rp[v]; e < G->rp[v + 1]; ++e)
        if (S->d[G->col[e]] == S->d[v] + G->w[e]) asum++;
    }
  }
  if (cnt) {
    cnt->n_s = (uint64_t)settled;
    cnt->m_s = msum;
    cnt->a_s = asum;
  }
  return settled;
}

/* Eq.(4) for every settled vertex, latest-settled first. */
static void backward(const og *G, oscratch *S, int64_t settled) {
  for (int64_t i = 0; i < settled; ++i) S->delta[S->order[i]] = 0.0L;
  for (int64_t i = settled - 1; i >= 0; --i) {
    int32_t v = S->order[i];
    long double acc = 0.0L;
    for (int64_t e = G->rp[v]; e < G->rp[v + 1]; ++e) {
      int32_t w = G->col[e];
      uint64_t len = G->w ? G->w[e] : 1;
      if (S->d[w] != OR_INF && S->d[w] == S->d[v] + len)
        acc += (long double)S->sigma[v] / (long double)S->sigma[w] * (1.0L + S->delta[w]);
    }
    S->delta[v] = acc;
  }
}

/* Full pass from s: distances (OR_INF unreached), sigma, delta_s.(v) for all
   v (0 where unreached, and delta_s.(s) as Eq.(4) gives it). */
int oracle_source_pass(int64_t n, int64_t m, const int64_t *rp, const int32_t *col,
                       const uint32_t *w, int32_t s, uint64_t *dist, uint64_t *sigma,
                       double *delta, int *overflow, uint64_t *counters) {
  if (s < 0 || s >= n || !overflow) return OR_INVALID;
  og G = {n, m, rp, col, w};
  oscratch S;
  if (scratch_init(&S, n, m) != OR_OK) { scratch_free(&S); return OR_NOMEM; }
  int ovf = 0;
  oc c;
  int64_t settled = forward(&G, s, &S, &ovf, &c);
  backward(&G, &S, settled);
  for (int64_t v = 0; v < n; ++v) {
    if (dist) dist[v] = S.d[v];
    if (sigma) sigma[v] = S.sigma[v];
    if (delta) delta[v] = S.d[v] == OR_INF ? 0.0 : (double)S.delta[v];
  }
  *overflow = ovf;
  if (counters) { counters[0] = c.n_s; counters[1] = c.m_s; counters[2] = c.a_s; }
  scratch_free(&S);
  return OR_OK;
}

/* ------------------------------------------------------- many sources
 * Each source s yields delta_s.(r_i) for every target r_i (0 for s = r_i,
 * which Eq.(3) excludes).  Sources run on worker threads; every result is
 * stored at its source's position, so the output does not depend on the
 * thread count. */

typedef struct {
  const og *G;
  const int32_t *src;
  int64_t ns;
  const int32_t *tgt;
  int64_t nt;
  double *res; /* [ns][nt] */
  oc *cnt;     /* [ns] or NULL */
  int64_t next;
  int ovf;
  int err;
  pthread_mutex_t mu;
} pool;

static void *worker(void *arg) {
  pool *P = arg;
  oscratch S;
  if (scratch_init(&S, P->G->n, P->G->m) != OR_OK) {
    scratch_free(&S);
    pthread_mutex_lock(&P->mu); P->err = OR_NOMEM; pthread_mutex_unlock(&P->mu);
    return NULL;
  }
  for (;;) {
    int64_t i = __atomic_fetch_add(&P->next, 1, __ATOMIC_RELAXED);
    if (i >= P->ns) break;
    int ovf = 0;
    oc c;
    int64_t settled = forward(P->G, P->src[i], &S, &ovf, &c);
    backward(P->G, &S, settled);
    for (int64_t j = 0; j < P->nt; ++j) {
      int32_t r = P->tgt[j];
      double v = 0.0;
      if (r != P->src[i] && S.d[r] != OR_INF) v = (double)S.delta[r];
      P->res[i * P->nt + j] = v;
    }
    if (P->cnt) P->cnt[i] = c;
    if (ovf) { pthread_mutex_lock(&P->mu); P->ovf = 1; pthread_mutex_unlock(&P->mu); }
  }
  scratch_free(&S);
  return NULL;
}

static int run_sources(const og *G, const int32_t *src, int64_t ns, const int32_t *tgt,
                       int64_t nt, int nthreads, double *res, oc *cnt, int *ovf) {
  pool P;
  memset(&P, 0, sizeof(P));
  P.G = G; P.src = src; P.ns = ns; P.tgt = tgt; P.nt = nt; P.res = res; P.cnt = cnt;
  pthread_mutex_init(&P.mu, NULL);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if (ns < nthreads) nthreads = ns > 0 ? (int)ns : 1;
  pthread_t th[256];
  int started = 0;
  for (int t = 1; t < nthreads; ++t)
    if (pthread_create(&th[started], NULL, worker, &P) == 0) started++;
  worker(&P);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&P.mu);
  *ovf = P.ovf;
  return P.err;
}

/* Neumaier-compensated sum in long double, in the given order */
static double comp_sum(const double *x, int64_t k, int64_t stride) {
  long double s = 0.0L, c = 0.0L;
  for (int64_t i = 0; i < k; ++i) {
    long double v = x[i * stride];
    long double t = s + v;
    if (fabsl(s) >= fabsl(v)) c += (s - t) + v;
    else c += (v - t) + s;
    s = t;
  }
  return (double)(s + c);
}

typedef struct {
  int64_t rv_size; /* -1: out-degree shortcut taken */
  int64_t fr_size;
  int64_t samples;
  int64_t distinct_sources;
  uint64_t te, reached, dag_arcs;
} ostats;

static void sum_counters(const oc *c, int64_t k, ostats *st) {
  st->te = st->reached = st->dag_arcs = 0;
  for (int64_t i = 0; i < k; ++i) {
    st->te += c[i].m_s;
    st->reached += c[i].n_s;
    st->dag_arcs += c[i].a_s;
  }
}

/* E-BCD, Alg.1.  pruned = 0 runs every source s != r instead of RV(r)
   (plain Brandes restricted to target r), for the Prop.1 invariant. */
int oracle_bc_exact(int64_t n, int64_t m, const int64_t *rp, const int32_t *col,
                    const uint32_t *w, int32_t r, int pruned, int nthreads, double *bc,
                    ostats *st) {
  if (r < 0 || r >= n || !bc) return OR_INVALID;
  og G = {n, m, rp, col, w};
  ostats local;
  memset(&local, 0, sizeof(local));
  if (rp[r + 1] == rp[r]) { /* Prop.1: out-degree 0 gives 0 */
    local.rv_size = -1;
    *bc = 0.0;
    if (st) *st = local;
    return OR_OK;
  }
  int32_t *src = malloc((size_t)n * sizeof(int32_t));
  if (!src) return OR_NOMEM;
  int64_t ns = 0;
  int rc = oracle_rv(n, m, rp, col, r, src, n, &ns);
  if (rc != OR_OK) { free(src); return rc; }
  local.rv_size = ns;
  if (!pruned) {
    ns = 0;
    for (int32_t v = 0; v < n; ++v)
      if (v != r) src[ns++] = v;
  }
  double *res = malloc((size_t)(ns ? ns : 1) * sizeof(double));
  oc *cnt = malloc((size_t)(ns ? ns : 1) * sizeof(oc));
  if (!res || !cnt) { free(src); free(res); free(cnt); return OR_NOMEM; }
  int ovf = 0;
  rc = run_sources(&G, src, ns, &r, 1, nthreads, res, cnt, &ovf);
  if (rc == OR_OK && ovf) rc = OR_OVERFLOW;
  if (rc == OR_OK) {
    *bc = comp_sum(res, ns, 1);
    local.distinct_sources = ns;
    sum_counters(cnt, ns, &local);
    if (st) *st = local;
  }
  free(src); free(res); free(cnt);
  return rc;
}

/* Per-source dependencies delta_s.(r) for an explicit source list (used by
   tests to compare source by source and by the CPU baseline timing). */
int oracle_dependencies(int64_t n, int64_t m, const int64_t *rp, const int32_t *col,
                        const uint32_t *w, int32_t r, const int32_t *src, int64_t ns,
                        int nthreads, double *dep, uint64_t *counters) {
  if (r < 0 || r >= n || (ns > 0 && (!src || !dep))) return OR_INVALID;
  for (int64_t i = 0; i < ns; ++i)
    if (src[i] < 0 || src[i] >= n) return OR_INVALID;
  og G = {n, m, rp, col, w};
  oc *cnt = malloc((size_t)(ns ? ns : 1) * sizeof(oc));
  if (!cnt) return OR_NOMEM;
  int ovf = 0;
  int rc = run_sources(&G, src, ns, &r, 1, nthreads, dep, cnt, &ovf);
  if (rc == OR_OK && ovf) rc = OR_OVERFLOW;
  if (counters)
    for (int64_t i = 0; i < ns; ++i) {
      counters[3 * i] = cnt[i].n_s;
      counters[3 * i + 1] = cnt[i].m_s;
      counters[3 * i + 2] = cnt[i].a_s;
    }
  free(cnt);
  return rc;
}

/* Set variant (Section 4.2): D = union of RV(r_i); one pass per s in D
   serves every r_i; BC(r_i) sums delta_s.(r_i) over s in D, s != r_i.  A
   target with out-degree 0 gets 0 (Prop.1).  Targets may repeat. */
int oracle_bc_set(int64_t n, int64_t m, const int64_t *rp, const int32_t *col,
                  const uint32_t *w, const int32_t *rs, int64_t l, int nthreads, double *bc,
                  ostats *st) {
  if (!rs || l <= 0 || !bc) return OR_INVALID;
  for (int64_t i = 0; i < l; ++i)
    if (rs[i] < 0 || rs[i] >= n) return OR_INVALID;
  og G = {n, m, rp, col, w};
  char *inD = calloc((size_t)n, 1);
  int32_t *tmp = malloc((size_t)n * sizeof(int32_t));
  if (!inD || !tmp) { free(inD); free(tmp); return OR_NOMEM; }
  for (int64_t i = 0; i < l; ++i) {
    int32_t r = rs[i];
    if (rp[r + 1] == rp[r]) continue;
    int64_t k = 0;
    int rc = oracle_rv(n, m, rp, col, r, tmp, n, &k);
    if (rc != OR_OK) { free(inD); free(tmp); return rc; }
    for (int64_t j = 0; j < k; ++j) inD[tmp[j]] = 1;
  }
  int64_t ns = 0;
  for (int32_t v = 0; v < n; ++v)
    if (inD[v]) tmp[ns++] = v;
  double *res = malloc((size_t)(ns ? ns : 1) * (size_t)l * sizeof(double));
  oc *cnt = malloc((size_t)(ns ? ns : 1) * sizeof(oc));
  if (!res || !cnt) { free(inD); free(tmp); free(res); free(cnt); return OR_NOMEM; }
  int ovf = 0;
  int rc = run_sources(&G, tmp, ns, rs, l, nthreads, res, cnt, &ovf);
  if (rc == OR_OK && ovf) rc = OR_OVERFLOW;
  if (rc == OR_OK) {
    for (int64_t i = 0; i < l; ++i) {
      int32_t r = rs[i];
      bc[i] = (rp[r + 1] == rp[r]) ? 0.0 : comp_sum(res + i, ns, l);
    }
    if (st) {
      memset(st, 0, sizeof(*st));
      st->rv_size = ns;
      st->distinct_sources = ns;
      sum_counters(cnt, ns, st);
    }
  }
  free(inD); free(tmp); free(res); free(cnt);
  return rc;
}

/* ---------------------------------------------------------- sampling
 * Draw t (t = 0, 1, ...) of a query with seed S: x = mix64(S + (t+1) G),
 * the t-th output of SplitMix64 (Steele, Lea, Flood 2014) started at S;
 * index = floor(x * |RV| / 2^64) into the ascending RV(r) list. */
static uint64_t o_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

int64_t oracle_draw_index(uint64_t seed, int64_t t, int64_t rv_size) {
  uint64_t x = o_mix64(seed + (uint64_t)(t + 1) * 0x9E3779B97F4A7C15ULL);
  return (int64_t)(((unsigned __int128)x * (unsigned __int128)(uint64_t)rv_size) >> 64);
}

/* Eq.(8): smallest integer T with T >= ln(2/delta) K^2 |RV|^2 / (2 eps^2),
   at least 1.  Saturates at INT64_MAX. */
int oracle_sample_count(double eps_abs, double delta, double K, int64_t rv_size, int64_t *T) {
  if (!(eps_abs > 0) || !(delta > 0 && delta < 1) || !(K >= 0) || rv_size < 0 || !T)
    return OR_INVALID;
  long double x = logl(2.0L / (long double)delta) * (long double)K * (long double)K *
                  (long double)rv_size * (long double)rv_size /
                  (2.0L * (long double)eps_abs * (long double)eps_abs);
  long double c = ceill(x);
  if (c < 1.0L) c = 1.0L;
  if (c >= 9.2e18L) *T = INT64_MAX;
  else *T = (int64_t)c;
  return OR_OK;
}

/* A-BCD, Alg.2, with T given: bc = |RV|/T * sum_t delta_{v_t}.(r).  Each
   distinct drawn source is computed once and reused for its repeats; the
   sum runs in draw order. */
int oracle_bc_sampled(int64_t n, int64_t m, const int64_t *rp, const int32_t *col,
                      const uint32_t *w, int32_t r, int64_t T, uint64_t seed, int nthreads,
                      double *bc, ostats *st) {
  if (r < 0 || r >= n || T <= 0 || !bc) return OR_INVALID;
  og G = {n, m, rp, col, w};
  ostats local;
  memset(&local, 0, sizeof(local));
  local.samples = T;
  if (rp[r + 1] == rp[r]) {
    local.rv_size = -1;
    *bc = 0.0;
    if (st) *st = local;
    return OR_OK;
  }
  int32_t *rv = malloc((size_t)n * sizeof(int32_t));
  if (!rv) return OR_NOMEM;
  int64_t k = 0;
  int rc = oracle_rv(n, m, rp, col, r, rv, n, &k);
  if (rc != OR_OK) { free(rv); return rc; }
  local.rv_size = k;
  if (k == 0) {
    *bc = 0.0;
    if (st) *st = local;
    free(rv);
    return OR_OK;
  }
  int64_t *slot = malloc((size_t)k * sizeof(int64_t));
  int64_t *draw = malloc((size_t)T * sizeof(int64_t));
  int32_t *uniq = malloc((size_t)(T < k ? T : k) * sizeof(int32_t));
  if (!slot || !draw || !uniq) { free(rv); free(slot); free(draw); free(uniq); return OR_NOMEM; }
  for (int64_t i = 0; i < k; ++i) slot[i] = -1;
  int64_t nu = 0;
  for (int64_t t = 0; t < T; ++t) {
    int64_t idx = oracle_draw_index(seed, t, k);
    if (slot[idx] < 0) { slot[idx] = nu; uniq[nu++] = rv[idx]; }
    draw[t] = slot[idx];
  }
  double *res = malloc((size_t)nu * sizeof(double));
  oc *cnt = malloc((size_t)nu * sizeof(oc));
  double *seq = malloc((size_t)T * sizeof(double));
  if (!res || !cnt || !seq) {
    free(rv); free(slot); free(draw); free(uniq); free(res); free(cnt); free(seq);
    return OR_NOMEM;
  }
  int ovf = 0;
  rc = run_sources(&G, uniq, nu, &r, 1, nthreads, res, cnt, &ovf);
  if (rc == OR_OK && ovf) rc = OR_OVERFLOW;
  if (rc == OR_OK) {
    for (int64_t t = 0; t < T; ++t) seq[t] = res[draw[t]];
    *bc = comp_sum(seq, T, 1) * (double)k / (double)T;
    local.distinct_sources = nu;
    sum_counters(cnt, nu, &local);
    if (st) *st = local;
  }
  free(rv); free(slot); free(draw); free(uniq); free(res); free(cnt); free(seq);
  return rc;
}

/* Baseline without the pruning (uniform source sampling over V, the
 * related-work estimator the paper compares its sample bound with after
 * Eq.(8)): draws index the ascending list V \ {r} with the same SplitMix64
 * rule; bc = (n-1)/T * sum_t delta_{v_t}.(r).  Unbiased because sources
 * outside RV(r) contribute 0 (Prop.1). */
int oracle_bc_sampled_all(int64_t n, int64_t m, const int64_t *rp, const int32_t *col, const uint32_t *w,
                          int32_t r, int64_t T, uint64_t seed, int nthreads, double *bc) {
  if (r < 0 || r >= n || T <= 0 || !bc || n < 2) return OR_INVALID;
  og G = {n, m, rp, col, w};
  if (rp[r + 1] == rp[r]) { *bc = 0.0; return OR_OK; }
  const int64_t k = n - 1;
  int64_t *draw = malloc((size_t)T * sizeof(int64_t));
  int32_t *uniq = malloc((size_t)T * sizeof(int32_t));
  int64_t *slot = malloc((size_t)k * sizeof(int64_t));
  if (!draw || !uniq || !slot) { free(draw); free(uniq); free(slot); return OR_NOMEM; }
  for (int64_t i = 0; i < k; ++i) slot[i] = -1;
  int64_t nu = 0;
  for (int64_t t = 0; t < T; ++t) {
    int64_t idx = oracle_draw_index(seed, t, k);
    if (slot[idx] < 0) {
      slot[idx] = nu;
      uniq[nu++] = (int32_t)(idx < r ? idx : idx + 1); /* idx-th vertex of V \ {r} */
    }
    draw[t] = slot[idx];
  }
  double *res = malloc((size_t)nu * sizeof(double));
  double *seq = malloc((size_t)T * sizeof(double));
  if (!res || !seq) { free(draw); free(uniq); free(slot); free(res); free(seq); return OR_NOMEM; }
  int ovf = 0;
  int rc = run_sources(&G, uniq, nu, &r, 1, nthreads, res, NULL, &ovf);
  if (rc == OR_OK && ovf) rc = OR_OVERFLOW;
  if (rc == OR_OK) {
    for (int64_t t = 0; t < T; ++t) seq[t] = res[draw[t]];
    *bc = comp_sum(seq, T, 1) * (double)k / (double)T;
  }
  free(draw); free(uniq); free(slot); free(res); free(seq);
  return rc;
}

/* ------------------------------------------------- definition, Eq.(1)
 * delta_s.(r) straight from the definition, without the Eq.(4) recursion:
 * a shortest s->t path passes through r iff d(s,r) + d(r,t) = d(s,t), and
 * then sigma_st(r) = sigma_sr * sigma_rt.  Needs one pass from s and one
 * from r.  (Only for checking the recursion; the paper gives Eq.(1)-(2).) */
int oracle_pair_dependency(int64_t n, int64_t m, const int64_t *rp, const int32_t *col,
                           const uint32_t *w, int32_t s, int32_t r, double *dep) {
  if (s < 0 || s >= n || r < 0 || r >= n || !dep) return OR_INVALID;
  og G = {n, m, rp, col, w};
  oscratch A, B;
  if (scratch_init(&A, n, m) != OR_OK || scratch_init(&B, n, m) != OR_OK) {
    scratch_free(&A); scratch_free(&B);
    return OR_NOMEM;
  }
  int ovf = 0;
  forward(&G, s, &A, &ovf, NULL);
  forward(&G, r, &B, &ovf, NULL);
  long double acc = 0.0L;
  if (s != r && A.d[r] != OR_INF) {
    for (int64_t t = 0; t < n; ++t) {
      if (t == s || t == r || A.d[t] == OR_INF || B.d[t] == OR_INF) continue;
      if (A.d[r] + B.d[t] == A.d[t])
        acc += (long double)A.sigma[r] * (long double)B.sigma[t] / (long double)A.sigma[t];
    }
  }
  *dep = (double)acc;
  scratch_free(&A); scratch_free(&B);
  return ovf ? OR_OVERFLOW : OR_OK;
}
