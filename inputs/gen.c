/*
 * Seeded synthetic inputs for the exponential-shift low-diameter decomposition.
 *
 * This module produces the two inputs the decomposition consumes and nothing else:
 *   - undirected graphs in CSR form (int32 row offsets and column ids, symmetric,
 *     no self-loops, no duplicate arcs, every adjacency list sorted ascending);
 *   - the per-vertex random shifts delta_u ~ Exp(beta) of Algorithm 1 step 1 (Sec. 2) and
 *     Algorithm 2 step 1 (Sec. 4), quantised to int64 fixed point with 20 fractional bits.
 * Both the CPU oracle and the GPU library read what this module writes; it holds none of
 * the decomposition's own arithmetic (no distances, no argmin, no cut counting).
 *
 * Randomness: one counter-based generator, SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014).  Draw i of stream s is the
 * SplitMix64 output for state s + (i+1)*0x9E3779B97F4A7C15, so every draw is a pure function
 * of (seed, purpose, index) and results do not depend on the thread count.
 *
 * Build: gcc -O3 -fopenmp -shared -fPIC gen.c -o libldd_inputs.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GOLDEN 0x9E3779B97F4A7C15ULL
#define FIX_ONE 1048576.0 /* 2^20: fixed-point scale of the shifts */

/* Purpose tags: each kind of draw gets its own stream so that inputs never share draws. */
enum { TAG_SHIFT = 1, TAG_RMAT = 2, TAG_RELABEL = 3, TAG_ER = 4, TAG_RGG = 5, TAG_PERM = 6 };

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Stream state for (seed, tag). */
uint64_t ldd_in_stream(uint64_t seed, uint64_t tag) {
  return mix64(mix64(seed + GOLDEN) ^ (tag * 0xD1B54A32D192ED03ULL));
}

/* Draw i of a stream: the SplitMix64 output after i+1 state increments. */
static inline uint64_t draw(uint64_t stream, uint64_t i) { return mix64(stream + (i + 1) * GOLDEN); }

/* Uniform double in [0,1) with 53 random bits. */
static inline double u01(uint64_t stream, uint64_t i) { return (double)(draw(stream, i) >> 11) * 0x1.0p-53; }

uint64_t ldd_in_draw(uint64_t seed, uint64_t tag, uint64_t i) { return draw(ldd_in_stream(seed, tag), i); }
double ldd_in_u01(uint64_t seed, uint64_t tag, uint64_t i) { return u01(ldd_in_stream(seed, tag), i); }

/* ------------------------------------------------------------------------------------------ */
/* Shifts: delta_u ~ Exp(beta) (rate beta, mean 1/beta; Sec. 3 density beta*exp(-beta x)),  */
/* sampled by inversion of the CDF 1 - exp(-beta x): delta = -ln(1 - U)/beta, U in [0,1),     */
/* quantised by truncation: shift_fix = floor(delta * 2^20).                                   */
/*                                                                                            */
/* The logarithm is evaluated with integers only, so that any implementation of this recipe  */
/* (CPU or GPU) gives the same bits: with U = (x >> 11) 2^-53 and M = 2^53 - (x >> 11), in    */
/* [1, 2^53], -ln(1-U) = ln 2 * (53 - log2 M).  log2 M = e + log2(m), e = floor(log2 M) and   */
/* m in [1, 2) held as a 64-bit fraction; the bits of log2(m) come from repeated squaring    */
/* (square m: if m^2 >= 2 the next bit is 1 and m becomes m^2 / 2, else it is 0 and m becomes */
/* m^2), 47 of them, truncated.  T = 2^47 (53 - e) - bits is an integer below 2^53, so it    */
/* converts to double exactly; then                                                            */
/*     shift_fix = floor( (T * (ln 2 * 2^-27)) / beta )                                        */
/* with one IEEE double multiplication and one division, each correctly rounded (the factor  */
/* ln 2 * 2^-27 folds 2^-47 of T and 2^20 of the fixed point into the constant ln 2).         */
/* ------------------------------------------------------------------------------------------ */
static inline uint64_t neglog2_q47(uint64_t x) {
  const uint64_t M = (1ULL << 53) - (x >> 11);
  const int e = 63 - __builtin_clzll(M);
  uint64_t m = M << (63 - e); /* m / 2^63 in [1, 2) */
  uint64_t bits = 0;
  for (int k = 0; k < 47; ++k) {
    const unsigned __int128 sq = (unsigned __int128)m * m; /* sq / 2^126 in [1, 4) */
    bits <<= 1;
    if (sq >> 127) {
      bits |= 1;
      m = (uint64_t)(sq >> 64);
    } else {
      m = (uint64_t)(sq >> 63);
    }
  }
  return ((uint64_t)(53 - e) << 47) - bits;
}

#define LN2_2M27 0x1.62e42fefa39efp-28 /* ln 2 * 2^-27 (the double nearest ln 2, scaled) */

int ldd_in_make_shifts(int64_t n, double beta, uint64_t seed, int64_t* out) {
  if (n < 0 || (out == NULL && n > 0) || !(beta > 0.0) || !isfinite(beta)) return 1;
  const uint64_t st = ldd_in_stream(seed, TAG_SHIFT);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const double t = (double)neglog2_q47(draw(st, (uint64_t)i));
    out[i] = (int64_t)floor((t * LN2_2M27) / beta);
  }
  return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Shift variants of the closing remarks of Sec. 5.                                           */
/*   kind 1 (integer shifts, permutation tie-break): the integer part of the Exp(beta) shift   */
/*     above (same draws), plus a fractional part that encodes a uniformly random ranking of  */
/*     the vertices -- rank 0 wins every tie: frac = floor((n - 1 - rank) 2^20 / n), distinct  */
/*     while n <= 2^20 (beyond, ranks 2^-20 apart share a fraction and the smaller id wins).  */
/*   kind 2 (shifts from permutation positions): the vertex of rank i takes the expected i-th */
/*     largest of n Exp(beta) draws, (H_n - H_i) / beta with H_i = sum_{j<=i} 1/j (Renyi's     */
/*     representation of exponential order statistics), so no exponential is sampled.         */
/*     The suffix sums S_i = sum_{j=i+1..n} 1/j are accumulated from S_n = 0 downwards in     */
/*     double; shift_fix = floor((S_i / beta) * 2^20).                                        */
/* The ranking sorts the vertices by a 64-bit draw of stream (seed, TAG_PERM), ties by id.     */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  uint64_t key;
  int64_t v;
} perm_item;

static int cmp_perm(const void* a, const void* b) {
  const perm_item *x = (const perm_item*)a, *y = (const perm_item*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return (x->v > y->v) - (x->v < y->v);
}

/* rank[v] in [0, n): position of v in the seeded random order */
static int perm_ranks(int64_t n, uint64_t seed, int64_t* rank) {
  perm_item* it = (perm_item*)malloc((size_t)(n > 0 ? n : 1) * sizeof(perm_item));
  if (!it) return 1;
  const uint64_t st = ldd_in_stream(seed, TAG_PERM);
  for (int64_t v = 0; v < n; ++v) {
    it[v].key = draw(st, (uint64_t)v);
    it[v].v = v;
  }
  qsort(it, (size_t)n, sizeof(perm_item), cmp_perm);
  for (int64_t i = 0; i < n; ++i) rank[it[i].v] = i;
  free(it);
  return 0;
}

int ldd_in_make_shifts_variant(int64_t n, double beta, uint64_t seed, int kind, int64_t* out) {
  if (kind == 0) return ldd_in_make_shifts(n, beta, seed, out);
  if (n < 0 || (out == NULL && n > 0) || !(beta > 0.0) || !isfinite(beta) || (kind != 1 && kind != 2)) return 1;
  if (n == 0) return 0;
  int64_t* rank = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  if (!rank || perm_ranks(n, seed, rank)) {
    free(rank);
    return 2;
  }
  if (kind == 1) {
    if (ldd_in_make_shifts(n, beta, seed, out)) {
      free(rank);
      return 1;
    }
    for (int64_t v = 0; v < n; ++v) {
      const int64_t frac = (int64_t)(((unsigned __int128)(n - 1 - rank[v]) << 20) / (unsigned __int128)n);
      out[v] = (out[v] >> 20 << 20) | frac;
    }
  } else {
    double* sfx = (double*)malloc((size_t)(n + 1) * sizeof(double));
    if (!sfx) {
      free(rank);
      return 2;
    }
    sfx[n] = 0.0;
    for (int64_t i = n - 1; i >= 0; --i) sfx[i] = sfx[i + 1] + 1.0 / (double)(i + 1);
    for (int64_t v = 0; v < n; ++v) out[v] = (int64_t)floor((sfx[rank[v]] / beta) * FIX_ONE);
    free(sfx);
  }
  free(rank);
  return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Graph container (malloc-owned; the caller copies out and frees).                           */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  int64_t n;
  int64_t nnz;
  int32_t* row_ptr; /* n+1 */
  int32_t* col_idx; /* nnz */
} ldd_in_graph;

void ldd_in_graph_free(ldd_in_graph* g) {
  if (!g) return;
  free(g->row_ptr);
  free(g->col_idx);
  free(g);
}
int64_t ldd_in_graph_n(const ldd_in_graph* g) { return g ? g->n : -1; }
int64_t ldd_in_graph_nnz(const ldd_in_graph* g) { return g ? g->nnz : -1; }
void ldd_in_graph_copy(const ldd_in_graph* g, int32_t* row_ptr, int32_t* col_idx) {
  memcpy(row_ptr, g->row_ptr, (size_t)(g->n + 1) * sizeof(int32_t));
  if (g->nnz) memcpy(col_idx, g->col_idx, (size_t)g->nnz * sizeof(int32_t));
}

static int cmp_i32(const void* a, const void* b) {
  const int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

static void sort_i32(int32_t* a, int64_t len) {
  if (len < 24) {
    for (int64_t i = 1; i < len; ++i) {
      int32_t v = a[i];
      int64_t j = i - 1;
      while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
      a[j + 1] = v;
    }
  } else {
    qsort(a, (size_t)len, sizeof(int32_t), cmp_i32);
  }
}

/*
 * Symmetric CSR from an undirected edge list: each pair (s,d) with s != d contributes the
 * arcs s->d and d->s; self-loops are dropped and repeated arcs are merged.  Returns NULL on
 * allocation failure or if the arc count does not fit int32 offsets.
 */
static ldd_in_graph* csr_from_pairs(int64_t n, int64_t m, const int32_t* src, const int32_t* dst) {
  ldd_in_graph* g = (ldd_in_graph*)calloc(1, sizeof(ldd_in_graph));
  int64_t* off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!g || !off) { free(g); free(off); return NULL; }
  g->n = n;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    const int32_t s = src[k], d = dst[k];
    if (s == d) continue;
#pragma omp atomic
    off[s + 1]++;
#pragma omp atomic
    off[d + 1]++;
  }
  for (int64_t v = 0; v < n; ++v) off[v + 1] += off[v];
  const int64_t raw = off[n];
  int32_t* buf = (int32_t*)malloc((size_t)(raw > 0 ? raw : 1) * sizeof(int32_t));
  int64_t* cur = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!buf || !cur) { free(buf); free(cur); free(off); free(g); return NULL; }
  memcpy(cur, off, (size_t)n * sizeof(int64_t));
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    const int32_t s = src[k], d = dst[k];
    if (s == d) continue;
    int64_t p, q;
#pragma omp atomic capture
    p = cur[s]++;
#pragma omp atomic capture
    q = cur[d]++;
    buf[p] = d;
    buf[q] = s;
  }
  free(cur);
  /* sort + unique each row in place; record the new degree */
  int64_t* deg = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!deg) { free(buf); free(off); free(g); return NULL; }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v) {
    int32_t* a = buf + off[v];
    const int64_t len = off[v + 1] - off[v];
    sort_i32(a, len);
    int64_t w = 0;
    for (int64_t i = 0; i < len; ++i)
      if (w == 0 || a[i] != a[w - 1]) a[w++] = a[i];
    deg[v] = w;
  }
  int64_t total = 0;
  for (int64_t v = 0; v < n; ++v) total += deg[v];
  if (total > INT32_MAX) { free(deg); free(buf); free(off); free(g); return NULL; }
  g->nnz = total;
  g->row_ptr = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
  g->col_idx = (int32_t*)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
  if (!g->row_ptr || !g->col_idx) { free(deg); free(buf); free(off); ldd_in_graph_free(g); return NULL; }
  g->row_ptr[0] = 0;
  for (int64_t v = 0; v < n; ++v) g->row_ptr[v + 1] = (int32_t)(g->row_ptr[v] + deg[v]);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v)
    memcpy(g->col_idx + g->row_ptr[v], buf + off[v], (size_t)deg[v] * sizeof(int32_t));
  free(deg);
  free(buf);
  free(off);
  return g;
}

ldd_in_graph* ldd_in_from_edges(int64_t n, int64_t m, const int32_t* src, const int32_t* dst) {
  if (n < 0 || n > INT32_MAX || m < 0) return NULL;
  for (int64_t k = 0; k < m; ++k)
    if (src[k] < 0 || src[k] >= n || dst[k] < 0 || dst[k] >= n) return NULL;
  return csr_from_pairs(n, m, src, dst);
}

/* ------------------------------------------------------------------------------------------ */
/* Grids: 4-neighbour 2D (id = i*cols + j) and 6-neighbour 3D (id = (x*Y + y)*Z + z).        */
/* ------------------------------------------------------------------------------------------ */
ldd_in_graph* ldd_in_grid2d(int64_t rows, int64_t cols) {
  if (rows < 0 || cols < 0) return NULL;
  const int64_t n = rows * cols;
  const int64_t nnz = 2 * (rows * (cols > 0 ? cols - 1 : 0) + cols * (rows > 0 ? rows - 1 : 0));
  if (n > INT32_MAX || nnz > INT32_MAX) return NULL;
  ldd_in_graph* g = (ldd_in_graph*)calloc(1, sizeof(ldd_in_graph));
  if (!g) return NULL;
  g->n = n;
  g->nnz = nnz;
  g->row_ptr = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
  g->col_idx = (int32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
  if (!g->row_ptr || !g->col_idx) { ldd_in_graph_free(g); return NULL; }
  g->row_ptr[0] = 0;
  for (int64_t v = 0; v < n; ++v) {
    const int64_t i = v / cols, j = v % cols;
    g->row_ptr[v + 1] = g->row_ptr[v] + (i > 0) + (j > 0) + (j + 1 < cols) + (i + 1 < rows);
  }
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    const int64_t i = v / cols, j = v % cols;
    int32_t* a = g->col_idx + g->row_ptr[v];
    if (i > 0) *a++ = (int32_t)(v - cols);
    if (j > 0) *a++ = (int32_t)(v - 1);
    if (j + 1 < cols) *a++ = (int32_t)(v + 1);
    if (i + 1 < rows) *a++ = (int32_t)(v + cols);
  }
  return g;
}

ldd_in_graph* ldd_in_grid3d(int64_t X, int64_t Y, int64_t Z) {
  if (X < 0 || Y < 0 || Z < 0) return NULL;
  const int64_t n = X * Y * Z;
  if (n > INT32_MAX) return NULL;
  const int64_t und = (X > 0 ? X - 1 : 0) * Y * Z + X * (Y > 0 ? Y - 1 : 0) * Z + X * Y * (Z > 0 ? Z - 1 : 0);
  if (2 * und > INT32_MAX) return NULL;
  ldd_in_graph* g = (ldd_in_graph*)calloc(1, sizeof(ldd_in_graph));
  if (!g) return NULL;
  g->n = n;
  g->nnz = 2 * und;
  g->row_ptr = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
  g->col_idx = (int32_t*)malloc((size_t)(g->nnz > 0 ? g->nnz : 1) * sizeof(int32_t));
  if (!g->row_ptr || !g->col_idx) { ldd_in_graph_free(g); return NULL; }
  g->row_ptr[0] = 0;
  for (int64_t v = 0; v < n; ++v) {
    const int64_t x = v / (Y * Z), y = (v / Z) % Y, z = v % Z;
    g->row_ptr[v + 1] = g->row_ptr[v] + (x > 0) + (y > 0) + (z > 0) + (z + 1 < Z) + (y + 1 < Y) + (x + 1 < X);
  }
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    const int64_t x = v / (Y * Z), y = (v / Z) % Y, z = v % Z;
    int32_t* a = g->col_idx + g->row_ptr[v];
    if (x > 0) *a++ = (int32_t)(v - Y * Z);
    if (y > 0) *a++ = (int32_t)(v - Z);
    if (z > 0) *a++ = (int32_t)(v - 1);
    if (z + 1 < Z) *a++ = (int32_t)(v + 1);
    if (y + 1 < Y) *a++ = (int32_t)(v + Z);
    if (x + 1 < X) *a++ = (int32_t)(v + Y * Z);
  }
  return g;
}

/* ------------------------------------------------------------------------------------------ */
/* RMAT / Kronecker: each of edgefactor*2^scale tuples descends `scale` levels of the 2x2     */
/* probability matrix [[a,b],[c,d]] (d = 1-a-b-c), one 32-bit uniform per level.  Optionally  */
/* vertex ids are relabelled by a seeded bijection of [0, 2^scale) so that hubs are not       */
/* clustered at small ids.  The result is symmetrised, self-loops dropped, duplicates merged. */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  uint64_t mul1, mul2, add1, add2;
  int bits;
  uint64_t mask;
} relabel_key;

static relabel_key make_relabel(int bits, uint64_t seed) {
  relabel_key k;
  const uint64_t st = ldd_in_stream(seed, TAG_RELABEL);
  k.bits = bits;
  k.mask = bits >= 64 ? ~0ULL : ((1ULL << bits) - 1);
  k.mul1 = draw(st, 0) | 1ULL; /* odd multipliers are bijections modulo 2^bits */
  k.mul2 = draw(st, 1) | 1ULL;
  k.add1 = draw(st, 2);
  k.add2 = draw(st, 3);
  return k;
}

/* A bijection of [0, 2^bits): alternating odd multiplications, additions and xor-shifts,
 * each of which is invertible modulo 2^bits. */
static inline uint64_t relabel(const relabel_key* k, uint64_t x) {
  const int h = k->bits / 2 > 0 ? k->bits / 2 : 1;
  for (int round = 0; round < 2; ++round) {
    x = (x * k->mul1 + k->add1) & k->mask;
    x ^= x >> h;
    x = (x * k->mul2 + k->add2) & k->mask;
    x ^= x >> (h > 1 ? h - 1 : 1);
  }
  return x & k->mask;
}

ldd_in_graph* ldd_in_rmat(int scale, int64_t edgefactor, double a, double b, double c, uint64_t seed,
                          int do_relabel) {
  if (scale < 1 || scale > 30 || edgefactor < 1) return NULL;
  if (!(a >= 0 && b >= 0 && c >= 0 && a + b + c <= 1.0)) return NULL;
  const int64_t n = (int64_t)1 << scale;
  const int64_t m = edgefactor * n;
  int32_t* src = (int32_t*)malloc((size_t)m * sizeof(int32_t));
  int32_t* dst = (int32_t*)malloc((size_t)m * sizeof(int32_t));
  if (!src || !dst) { free(src); free(dst); return NULL; }
  /* thresholds on a 32-bit uniform */
  const uint64_t ta = (uint64_t)floor(a * 4294967296.0);
  const uint64_t tab = (uint64_t)floor((a + b) * 4294967296.0);
  const uint64_t tabc = (uint64_t)floor((a + b + c) * 4294967296.0);
  const uint64_t st = ldd_in_stream(seed, TAG_RMAT);
  const uint64_t words = (uint64_t)(scale + 1) / 2; /* two 32-bit uniforms per draw */
  relabel_key rk = make_relabel(scale, seed);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint64_t s = 0, d = 0;
    for (int lvl = 0; lvl < scale; ++lvl) {
      const uint64_t w = draw(st, (uint64_t)e * words + (uint64_t)(lvl >> 1));
      const uint64_t r = (lvl & 1) ? (w >> 32) : (w & 0xFFFFFFFFULL);
      const uint64_t bs = r >= tab;                  /* quadrants c and d: lower half */
      const uint64_t bd = (r >= ta && r < tab) || r >= tabc; /* quadrants b and d: right half */
      s = (s << 1) | bs;
      d = (d << 1) | bd;
    }
    if (do_relabel) {
      s = relabel(&rk, s);
      d = relabel(&rk, d);
    }
    src[e] = (int32_t)s;
    dst[e] = (int32_t)d;
  }
  ldd_in_graph* g = csr_from_pairs(n, m, src, dst);
  free(src);
  free(dst);
  return g;
}

/* ------------------------------------------------------------------------------------------ */
/* Erdos-Renyi G(n,p): geometric skipping over the pairs (w < v) in row-major order, the      */
/* method of Batagelj and Brandes ("Efficient generation of large random networks", 2005).    */
/* ------------------------------------------------------------------------------------------ */
ldd_in_graph* ldd_in_er(int64_t n, double p, uint64_t seed) {
  if (n < 0 || n > INT32_MAX || !(p >= 0.0 && p <= 1.0)) return NULL;
  const uint64_t st = ldd_in_stream(seed, TAG_ER);
  int64_t cap = 1024, m = 0;
  int32_t* src = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
  int32_t* dst = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
  if (!src || !dst) { free(src); free(dst); return NULL; }
  if (p > 0.0 && n > 1) {
    const double lq = log1p(-p);
    int64_t v = 1, w = -1;
    uint64_t i = 0;
    while (v < n) {
      const double u = u01(st, i++);
      const double skip = (p >= 1.0) ? 0.0 : floor(log1p(-u) / lq);
      w += 1 + (int64_t)skip;
      while (w >= v && v < n) { w -= v; ++v; }
      if (v < n) {
        if (m == cap) {
          cap *= 2;
          int32_t* s2 = (int32_t*)realloc(src, (size_t)cap * sizeof(int32_t));
          int32_t* d2 = (int32_t*)realloc(dst, (size_t)cap * sizeof(int32_t));
          if (!s2 || !d2) { free(s2 ? s2 : src); free(d2 ? d2 : dst); return NULL; }
          src = s2;
          dst = d2;
        }
        src[m] = (int32_t)v;
        dst[m] = (int32_t)w;
        ++m;
      }
    }
  }
  ldd_in_graph* g = csr_from_pairs(n, m, src, dst);
  free(src);
  free(dst);
  return g;
}

/* ------------------------------------------------------------------------------------------ */
/* 2D random geometric graph: n points uniform in the unit square, an edge between every      */
/* pair at Euclidean distance <= r.  Points are bucketed into square cells of side >= r.      */
/* ------------------------------------------------------------------------------------------ */
ldd_in_graph* ldd_in_rgg(int64_t n, double r, uint64_t seed) {
  if (n < 0 || n > INT32_MAX || !(r > 0.0)) return NULL;
  const uint64_t st = ldd_in_stream(seed, TAG_RGG);
  double* x = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double* y = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  int64_t cells = (int64_t)floor(1.0 / r);
  if (cells < 1) cells = 1;
  if (cells > 65536) cells = 65536;
  const int64_t nc = cells * cells;
  int64_t* cstart = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
  int32_t* order = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int64_t* cellof = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!x || !y || !cstart || !order || !cellof) {
    free(x); free(y); free(cstart); free(order); free(cellof);
    return NULL;
  }
  for (int64_t i = 0; i < n; ++i) {
    x[i] = u01(st, 2 * (uint64_t)i);
    y[i] = u01(st, 2 * (uint64_t)i + 1);
    int64_t cx = (int64_t)(x[i] * cells), cy = (int64_t)(y[i] * cells);
    if (cx >= cells) cx = cells - 1;
    if (cy >= cells) cy = cells - 1;
    cellof[i] = cx * cells + cy;
    cstart[cellof[i] + 1]++;
  }
  for (int64_t k = 0; k < nc; ++k) cstart[k + 1] += cstart[k];
  {
    int64_t* cur = (int64_t*)malloc((size_t)nc * sizeof(int64_t));
    if (!cur) { free(x); free(y); free(cstart); free(order); free(cellof); return NULL; }
    memcpy(cur, cstart, (size_t)nc * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) order[cur[cellof[i]]++] = (int32_t)i;
    free(cur);
  }
  const double r2 = r * r;
  /* pass 1: degrees; pass 2: fill (each row then sorted) */
  int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!deg) { free(x); free(y); free(cstart); free(order); free(cellof); return NULL; }
  ldd_in_graph* g = (ldd_in_graph*)calloc(1, sizeof(ldd_in_graph));
  for (int pass = 0; pass < 2 && g; ++pass) {
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
      const int64_t cx = cellof[i] / cells, cy = cellof[i] % cells;
      int64_t cnt = 0;
      int32_t* out = pass ? g->col_idx + g->row_ptr[i] : NULL;
      for (int64_t dx = -1; dx <= 1; ++dx)
        for (int64_t dy = -1; dy <= 1; ++dy) {
          const int64_t ax = cx + dx, ay = cy + dy;
          if (ax < 0 || ay < 0 || ax >= cells || ay >= cells) continue;
          const int64_t k = ax * cells + ay;
          for (int64_t t = cstart[k]; t < cstart[k + 1]; ++t) {
            const int32_t j = order[t];
            if (j == i) continue;
            const double ex = x[i] - x[j], ey = y[i] - y[j];
            if (ex * ex + ey * ey <= r2) {
              if (pass) out[cnt] = j;
              ++cnt;
            }
          }
        }
      if (pass)
        sort_i32(out, cnt);
      else
        deg[i] = cnt;
    }
    if (pass == 0) {
      int64_t total = 0;
      for (int64_t i = 0; i < n; ++i) total += deg[i];
      if (total > INT32_MAX) { free(g); g = NULL; break; }
      g->n = n;
      g->nnz = total;
      g->row_ptr = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
      g->col_idx = (int32_t*)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
      if (!g->row_ptr || !g->col_idx) { ldd_in_graph_free(g); g = NULL; break; }
      g->row_ptr[0] = 0;
      for (int64_t i = 0; i < n; ++i) g->row_ptr[i + 1] = (int32_t)(g->row_ptr[i] + deg[i]);
    }
  }
  free(deg); free(x); free(y); free(cstart); free(order); free(cellof);
  return g;
}
