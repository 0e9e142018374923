/*
 * CPU ORACLE for the exponential-shift low-diameter decomposition -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the package smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code with the GPU library: it is plain, single-threaded
 * and written for obvious correctness, not speed.
 *
 * What it computes (Algorithm 2, Sec. 4, with the shifted distance of Eq. (1), Sec. 3):
 * each vertex v joins the centre u minimising  dist(u,v) - delta_u,  ties broken by the
 * smaller vertex id ("lexicographically").  Shifts arrive as int64 fixed point with 20
 * fractional bits, shift_fix[u] = floor(delta_u * 2^20), so every comparison is exact:
 *
 *     centre(v) = argmin_u  ( 2^20 * dist(u,v) - shift_fix[u] ,  u )   (lexicographic pair)
 *
 * over the vertices u in v's connected component (dist is infinite across components).
 * cut = number of undirected edges whose endpoints have different centres (Def. 1.1).
 *
 * Entry points
 *   oracle_decompose  whole graph, by the super-source shortest-path formulation of Sec. 5:
 *                     a source s with an arc of length (Delta - shift_fix[u]) to every u
 *                     (Delta = max shift, added so that lengths are non-negative) and unit
 *                     graph edges of length 2^20; v's piece is the first vertex after s on
 *                     its shortest path.  Solved with Dijkstra over (length, first-vertex)
 *                     pairs in lexicographic order, using an indexed binary heap.
 *   oracle_centre_of  one vertex, by the definition itself: breadth-first search from v
 *                     gives dist(u,v) for every u; take the lexicographic argmin.
 *   oracle_cut        cut edges of a given assignment (Def. 1.1).
 *   oracle_certify    linear-time check that a given assignment is the exact argmin, for
 *                     graphs too large for oracle_decompose in a test's time budget.
 *
 * Build: gcc -O2 -shared -fPIC ldd_oracle.c -o liblddoracle.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define S_ONE ((int64_t)1 << 20) /* one unit of graph distance in shift units */

enum {
  OR_OK = 0,
  OR_BAD_ARG = 1,
  OR_NO_MEM = 2,
  /* certificate failures */
  OR_BAD_CENTRE = 10,    /* centre id out of range, or a centre not its own centre */
  OR_DISCONNECTED = 11,  /* a vertex not reachable from its centre inside its piece */
  OR_NOT_MINIMAL_SELF = 12, /* a vertex would rather be its own centre */
  OR_NOT_MINIMAL_EDGE = 13  /* a vertex would rather join a neighbour's piece */
};

/*
 * Planted mistakes, used only by the tests that show the oracle's pins catch errors.
 * 0 is the oracle itself.
 */
enum {
  MUT_NONE = 0,
  MUT_TIE_LARGER_ID = 1,   /* equal shifted distance: larger id wins */
  MUT_SHIFT_SIGN = 2,      /* dist + delta instead of dist - delta */
  MUT_EDGE_LENGTH = 3,     /* edges one fixed-point unit too long */
  MUT_INTEGER_SHIFTS = 4,  /* fractional part of the shifts ignored */
  MUT_NO_TIEBREAK = 5      /* first label found kept on equal distance (no id order) */
};

static int valid_csr(int64_t n, const int32_t* row_ptr, const int32_t* col_idx) {
  if (n < 0 || n > INT32_MAX || (n > 0 && (!row_ptr || !col_idx))) return 0;
  if (n == 0) return 1;
  if (row_ptr[0] != 0) return 0;
  for (int64_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) return 0;
  for (int64_t a = 0; a < row_ptr[n]; ++a)
    if (col_idx[a] < 0 || col_idx[a] >= n) return 0;
  return 1;
}

static int valid_shifts(int64_t n, const int64_t* shift_fix) {
  for (int64_t v = 0; v < n; ++v)
    if (shift_fix[v] < 0 || shift_fix[v] > ((int64_t)1 << 52)) return 0;
  return 1;
}

int64_t oracle_cut(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const int32_t* centre);

/* lexicographic (length, first vertex) order */
static inline int lex_less(int64_t ka, int32_t oa, int64_t kb, int32_t ob) {
  return ka < kb || (ka == kb && oa < ob);
}

/* ---------------------------------------------------------------------------------------- */
/* Indexed binary min-heap over vertices, keyed by (len[v], org[v]).                         */
/* ---------------------------------------------------------------------------------------- */
typedef struct {
  int32_t* heap; /* heap[i] = vertex */
  int64_t* pos;  /* pos[v] = index in heap, -1 once removed */
  int64_t size;
  const int64_t* len;
  const int32_t* org;
  int mutation;
} heap_t;

static inline int h_less(const heap_t* h, int32_t a, int32_t b) {
  if (h->mutation == MUT_TIE_LARGER_ID)
    return h->len[a] < h->len[b] || (h->len[a] == h->len[b] && h->org[a] > h->org[b]);
  return lex_less(h->len[a], h->org[a], h->len[b], h->org[b]);
}

static inline void h_swap(heap_t* h, int64_t i, int64_t j) {
  const int32_t a = h->heap[i], b = h->heap[j];
  h->heap[i] = b;
  h->heap[j] = a;
  h->pos[b] = i;
  h->pos[a] = j;
}

static void h_up(heap_t* h, int64_t i) {
  while (i > 0) {
    const int64_t p = (i - 1) / 2;
    if (!h_less(h, h->heap[i], h->heap[p])) break;
    h_swap(h, i, p);
    i = p;
  }
}

static void h_down(heap_t* h, int64_t i) {
  for (;;) {
    const int64_t l = 2 * i + 1, r = l + 1;
    int64_t s = i;
    if (l < h->size && h_less(h, h->heap[l], h->heap[s])) s = l;
    if (r < h->size && h_less(h, h->heap[r], h->heap[s])) s = r;
    if (s == i) break;
    h_swap(h, i, s);
    i = s;
  }
}

static int32_t h_pop(heap_t* h) {
  const int32_t top = h->heap[0];
  h_swap(h, 0, h->size - 1);
  h->size--;
  h->pos[top] = -1;
  if (h->size > 0) h_down(h, 0);
  return top;
}

/* ---------------------------------------------------------------------------------------- */
int oracle_decompose_mut(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const int64_t* shift_fix,
                         int32_t* centre, int64_t* len_out, int64_t* cut_out, int mutation) {
  if (!valid_csr(n, row_ptr, col_idx) || (n > 0 && (!shift_fix || !centre))) return OR_BAD_ARG;
  if (!valid_shifts(n, shift_fix)) return OR_BAD_ARG;
  if (n == 0) {
    if (cut_out) *cut_out = 0;
    return OR_OK;
  }
  const int64_t edge_len = (mutation == MUT_EDGE_LENGTH) ? S_ONE + 1 : S_ONE;

  /* shift of each vertex as the algorithm sees it */
  int64_t* shift = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* len = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int32_t* org = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* heap = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int64_t* pos = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  if (!shift || !len || !org || !heap || !pos) {
    free(shift); free(len); free(org); free(heap); free(pos);
    return OR_NO_MEM;
  }
  for (int64_t u = 0; u < n; ++u) {
    int64_t s = shift_fix[u];
    if (mutation == MUT_INTEGER_SHIFTS) s = (s / S_ONE) * S_ONE;
    if (mutation == MUT_SHIFT_SIGN) s = -s;
    shift[u] = s;
  }

  /* Delta = max shift (Algorithm 1, step 2); source arc s->u has length Delta - shift[u] */
  int64_t delta = shift[0];
  for (int64_t u = 1; u < n; ++u)
    if (shift[u] > delta) delta = shift[u];

  /* tentative labels: the direct arc from the super source */
  for (int64_t u = 0; u < n; ++u) {
    len[u] = delta - shift[u];
    org[u] = (int32_t)u;
  }

  heap_t h = {heap, pos, n, len, org, mutation};
  for (int64_t i = 0; i < n; ++i) {
    heap[i] = (int32_t)i;
    pos[i] = i;
  }
  for (int64_t i = n / 2 - 1; i >= 0; --i) h_down(&h, i);

  /* Dijkstra: settle the smallest label, relax its graph edges */
  while (h.size > 0) {
    const int32_t v = h_pop(&h);
    const int64_t cand_len = len[v] + edge_len;
    const int32_t cand_org = org[v];
    for (int32_t a = row_ptr[v]; a < row_ptr[v + 1]; ++a) {
      const int32_t w = col_idx[a];
      if (pos[w] < 0) continue; /* already settled */
      int better;
      if (mutation == MUT_NO_TIEBREAK)
        better = cand_len < len[w];
      else if (mutation == MUT_TIE_LARGER_ID)
        better = cand_len < len[w] || (cand_len == len[w] && cand_org > org[w]);
      else
        better = lex_less(cand_len, cand_org, len[w], org[w]);
      if (better) {
        len[w] = cand_len;
        org[w] = cand_org;
        h_up(&h, pos[w]);
      }
    }
  }

  for (int64_t v = 0; v < n; ++v) centre[v] = org[v];
  if (len_out)
    for (int64_t v = 0; v < n; ++v) len_out[v] = len[v];
  if (cut_out) {
    int64_t cut_arcs = 0;
    for (int64_t v = 0; v < n; ++v)
      for (int32_t a = row_ptr[v]; a < row_ptr[v + 1]; ++a) cut_arcs += (org[col_idx[a]] != org[v]);
    *cut_out = cut_arcs / 2;
  }
  free(shift); free(len); free(org); free(heap); free(pos);
  return OR_OK;
}

/* centre[v] for every v; len_out (optional) receives Delta + min shifted distance in
 * fixed point; cut_out (optional) the number of cut undirected edges. */
int oracle_decompose(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const int64_t* shift_fix,
                     int32_t* centre, int64_t* len_out, int64_t* cut_out) {
  return oracle_decompose_mut(n, row_ptr, col_idx, shift_fix, centre, len_out, cut_out, MUT_NONE);
}

/* ---------------------------------------------------------------------------------------- */
/* The same result by the bucketed search of Sec. 5: lengths are processed one integer       */
/* distance ("round") at a time, with one bucket per integer part (Dial's bucket queue).     */
/* Vertex u's own source arc has length off[u] = Delta - shift[u] and enters at round        */
/* off[u] >> 20; a graph edge adds one unit (2^20), so a label first reached in round r      */
/* carries a length in [r 2^20, (r+1) 2^20).  Round r takes every own arc of its bucket and  */
/* every offer relayed from a vertex settled in round r-1, keeps per vertex the              */
/* lexicographically smallest (length, first vertex) pair, settles every vertex touched,     */
/* and relays the settled labels plus one unit to unsettled neighbours for round r+1.  Only  */
/* round r-1 can relay lengths of integer part r, so each round's minimum is final.          */
/* ---------------------------------------------------------------------------------------- */
int oracle_decompose_rounds(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const int64_t* shift_fix,
                            int32_t* centre, int64_t* len_out, int64_t* cut_out) {
  if (!valid_csr(n, row_ptr, col_idx) || (n > 0 && (!shift_fix || !centre))) return OR_BAD_ARG;
  if (!valid_shifts(n, shift_fix)) return OR_BAD_ARG;
  if (n == 0) {
    if (cut_out) *cut_out = 0;
    return OR_OK;
  }
  int64_t delta = 0;
  for (int64_t u = 0; u < n; ++u)
    if (shift_fix[u] > delta) delta = shift_fix[u];
  const int64_t rounds = (delta >> 20) + 1; /* own arcs enter in rounds 0 .. rounds-1 */
  int64_t* len = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int32_t* org = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int64_t* done = (int64_t*)malloc((size_t)n * sizeof(int64_t)); /* round settled, -1 = not yet */
  int64_t* bstart = (int64_t*)calloc((size_t)rounds + 1, sizeof(int64_t));
  int32_t* bucket = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* touched = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* settled = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  if (!len || !org || !done || !bstart || !bucket || !touched || !settled) {
    free(len); free(org); free(done); free(bstart); free(bucket); free(touched); free(settled);
    return OR_NO_MEM;
  }
  /* bucket of each own arc by the integer part of its length (counting sort) */
  for (int64_t u = 0; u < n; ++u) bstart[((delta - shift_fix[u]) >> 20) + 1]++;
  for (int64_t r = 0; r < rounds; ++r) bstart[r + 1] += bstart[r];
  for (int64_t u = 0; u < n; ++u) {
    const int64_t r = (delta - shift_fix[u]) >> 20;
    bucket[bstart[r]++] = (int32_t)u;
  }
  for (int64_t r = rounds; r > 0; --r) bstart[r] = bstart[r - 1];
  bstart[0] = 0;
  for (int64_t v = 0; v < n; ++v) {
    done[v] = -1;
    len[v] = INT64_MAX;
    org[v] = -1;
  }
  /* touched[0 .. nt) : vertices holding an offer for the current round (from relays) */
  int64_t nt = 0, left = n;
  for (int64_t r = 0; left > 0; ++r) {
    /* own arcs of bucket r compete with the relayed offers already in len / org */
    if (r < rounds)
      for (int64_t i = bstart[r]; i < bstart[r + 1]; ++i) {
        const int32_t u = bucket[i];
        if (done[u] >= 0) continue;
        const int64_t l = delta - shift_fix[u];
        if (org[u] < 0) touched[nt++] = u; /* first offer this round */
        if (lex_less(l, u, len[u], org[u] < 0 ? INT32_MAX : org[u])) {
          len[u] = l;
          org[u] = u;
        }
      }
    /* settle every touched vertex: its minimum over this round's offers is final */
    int64_t ns = 0;
    for (int64_t i = 0; i < nt; ++i) {
      const int32_t v = touched[i];
      done[v] = r;
      settled[ns++] = v;
    }
    left -= ns;
    nt = 0;
    /* relay to unsettled neighbours: offers for round r+1 */
    for (int64_t i = 0; i < ns; ++i) {
      const int32_t v = settled[i];
      const int64_t l = len[v] + S_ONE;
      for (int32_t a = row_ptr[v]; a < row_ptr[v + 1]; ++a) {
        const int32_t w = col_idx[a];
        if (done[w] >= 0) continue;
        if (org[w] < 0) {
          touched[nt++] = w;
          len[w] = l;
          org[w] = org[v];
        } else if (lex_less(l, org[v], len[w], org[w])) {
          len[w] = l;
          org[w] = org[v];
        }
      }
    }
  }
  for (int64_t v = 0; v < n; ++v) centre[v] = org[v];
  if (len_out)
    for (int64_t v = 0; v < n; ++v) len_out[v] = len[v];
  if (cut_out) *cut_out = oracle_cut(n, row_ptr, col_idx, centre);
  free(len); free(org); free(done); free(bstart); free(bucket); free(touched); free(settled);
  return OR_OK;
}

/* ---------------------------------------------------------------------------------------- */
/* The definition for one vertex: BFS from v gives dist(u,v) = dist(v,u) (undirected); the  */
/* centre is the lexicographic argmin of (2^20*dist(u,v) - shift_fix[u], u).  The search     */
/* stops once 2^20*d - max_shift exceeds the best value found, since no vertex at distance  */
/* d or more can then do better.                                                             */
/* ---------------------------------------------------------------------------------------- */
int oracle_centre_of(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const int64_t* shift_fix,
                     int64_t v, int32_t* centre_out, int64_t* shifted_out) {
  if (n <= 0 || v < 0 || v >= n || !row_ptr || !col_idx || !shift_fix || !centre_out) return OR_BAD_ARG;
  int64_t max_shift = 0;
  for (int64_t u = 0; u < n; ++u)
    if (shift_fix[u] > max_shift) max_shift = shift_fix[u];
  int32_t* dist = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* queue = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  if (!dist || !queue) { free(dist); free(queue); return OR_NO_MEM; }
  for (int64_t u = 0; u < n; ++u) dist[u] = -1;
  int64_t head = 0, tail = 0;
  dist[v] = 0;
  queue[tail++] = (int32_t)v;
  int64_t best = -shift_fix[v];
  int32_t best_u = (int32_t)v;
  while (head < tail) {
    const int32_t u = queue[head++];
    const int64_t val = S_ONE * dist[u] - shift_fix[u];
    if (val < best || (val == best && u < best_u)) {
      best = val;
      best_u = u;
    }
    if (S_ONE * (int64_t)(dist[u] + 1) - max_shift > best) continue; /* farther vertices cannot win */
    for (int32_t a = row_ptr[u]; a < row_ptr[u + 1]; ++a) {
      const int32_t w = col_idx[a];
      if (dist[w] < 0) {
        dist[w] = dist[u] + 1;
        queue[tail++] = w;
      }
    }
  }
  *centre_out = best_u;
  if (shifted_out) *shifted_out = best;
  free(dist);
  free(queue);
  return OR_OK;
}

/* Number of undirected edges {v,w} with centre[v] != centre[w] (Def. 1.1); each edge is
 * stored as two arcs, so the arc count is halved. */
int64_t oracle_cut(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const int32_t* centre) {
  int64_t arcs = 0;
  for (int64_t v = 0; v < n; ++v)
    for (int32_t a = row_ptr[v]; a < row_ptr[v + 1]; ++a) arcs += (centre[col_idx[a]] != centre[v]);
  return arcs / 2;
}

/* ---------------------------------------------------------------------------------------- */
/* Certificate of exactness for an assignment `centre`.                                      */
/*   L(v) = (Delta - shift[c(v)] + 2^20 * d_piece(c(v), v),  c(v))                           */
/* where d_piece is the BFS distance from the centre using only vertices of the piece.       */
/* L(v) is realised by a real path, so L(v) >= the exact minimum M(v).  If also              */
/*   (a) L(v) <= (Delta - shift[v], v)           for every v, and                            */
/*   (b) L(v) <= (L(w).len + 2^20, L(w).centre)   for every arc v-w,                         */
/* then along any path u = x0 .. xk = v, L(v) <= (Delta - shift[u] + 2^20 k, u), so          */
/* L(v) <= M(v) and the assignment is the exact lexicographic argmin.                        */
/* Returns OR_OK or the first failure kind; *bad receives the offending vertex.              */
/* ---------------------------------------------------------------------------------------- */
int oracle_certify(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const int64_t* shift_fix,
                   const int32_t* centre, int64_t* bad) {
  int64_t dummy;
  if (!bad) bad = &dummy;
  *bad = -1;
  if (!valid_csr(n, row_ptr, col_idx) || (n > 0 && (!shift_fix || !centre))) return OR_BAD_ARG;
  if (n == 0) return OR_OK;
  for (int64_t v = 0; v < n; ++v) {
    const int32_t c = centre[v];
    if (c < 0 || c >= n || centre[c] != c) { *bad = v; return OR_BAD_CENTRE; }
  }
  int64_t delta = 0;
  for (int64_t u = 0; u < n; ++u)
    if (shift_fix[u] > delta) delta = shift_fix[u];
  int32_t* d = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* queue = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  if (!d || !queue) { free(d); free(queue); return OR_NO_MEM; }
  int64_t head = 0, tail = 0;
  for (int64_t v = 0; v < n; ++v) {
    d[v] = -1;
    if (centre[v] == v) {
      d[v] = 0;
      queue[tail++] = (int32_t)v;
    }
  }
  while (head < tail) {
    const int32_t u = queue[head++];
    for (int32_t a = row_ptr[u]; a < row_ptr[u + 1]; ++a) {
      const int32_t w = col_idx[a];
      if (d[w] < 0 && centre[w] == centre[u]) {
        d[w] = d[u] + 1;
        queue[tail++] = w;
      }
    }
  }
  int rc = OR_OK;
  for (int64_t v = 0; v < n && rc == OR_OK; ++v) {
    if (d[v] < 0) { *bad = v; rc = OR_DISCONNECTED; break; }
    const int32_t c = centre[v];
    const int64_t lv = delta - shift_fix[c] + S_ONE * d[v];
    if (lex_less(delta - shift_fix[v], (int32_t)v, lv, c)) { *bad = v; rc = OR_NOT_MINIMAL_SELF; break; }
  }
  for (int64_t v = 0; v < n && rc == OR_OK; ++v) {
    const int32_t c = centre[v];
    const int64_t lv = delta - shift_fix[c] + S_ONE * d[v];
    for (int32_t a = row_ptr[v]; a < row_ptr[v + 1]; ++a) {
      const int32_t w = col_idx[a];
      if (d[w] < 0) continue; /* reported by the loop above */
      const int64_t lw = delta - shift_fix[centre[w]] + S_ONE * d[w];
      if (lex_less(lw + S_ONE, centre[w], lv, c)) { *bad = v; rc = OR_NOT_MINIMAL_EDGE; break; }
    }
  }
  free(d);
  free(queue);
  return rc;
}
