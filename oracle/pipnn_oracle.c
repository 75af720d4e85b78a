/*
 * PiPNN FP64 reference oracle.
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the GPU path. Only
 * the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it. It shares no code, header, table or helper with the GPU library, and
 * the GPU library never calls it.
 *
 * Everything here is a plain, slow, direct transcription of what the paper
 * (arXiv 2602.21247, "PiPNN: Ultra-Scalable Graph-Based Nearest Neighbor
 * Indexing") defines, in FP64:
 *   - dissimilarity: squared L2 or negative inner product (Preliminaries);
 *   - residualized hashing and the sketch form of it (Sec. 3, the hashing
 *     equation and the Implementation paragraph);
 *   - HashPrune, both as the streaming Alg. 3 and as the closed form of the
 *     history-independence lemma (Supplement, proof of determinism);
 *   - Randomized Ball Carving with fanout (Alg. 5, Sec. 4.1);
 *   - the bi-directed k-NN leaf pick (Sec. 4.2, Supplement "k-NN leaf
 *     design space") and the All-to-All Prune leaf picker (Supplement,
 *     "Picking within Leaves");
 *   - RobustPrune, standard (Alg. 2) and lazy (Supplement "Optimizing
 *     RobustPrune");
 *   - BeamSearch (Alg. 1) and brute-force k-NN (Definition of k-NN search).
 * Beside the paper's method it holds the encoders of the reduced-precision
 * leaf-GEMM operands (bf16, fp16, OCP e4m3 with a per-point scale), written
 * from the published format definitions, and the leaf pick over such an
 * operand with FP64 rescoring of the nearest candidates.
 *
 * Readings of passages the paper leaves open (tie-breaks, the leader count,
 * the merge rule, the random stream) are fixed in the comments below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EMPTY_ID 0xFFFFFFFFu
#define ORC_BF16_INF 0x7F80u

typedef struct {
  int32_t metric; /* 0: squared L2, 1: negative inner product */
  int32_t c_max, c_min, leader_div, leader_cap;
  int32_t fanout[4];
  int32_t k, hash_bits, l_max, R;
  float alpha;
  int32_t pad_;
  uint64_t seed;
} orc_params;

int orc_version(void) { return 1; }

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Dissimilarity (Preliminaries): squared L2 by direct difference with the
 * coordinate index ascending, or the negated inner product. */
/* Wall time of each phase, summed over the calls since the last reset:
 * CLOCK_MONOTONIC (a steady clock) read at the entry and exit of every
 * exported phase function. Timing only; it never changes a result. */
enum {
  ORC_PH_SKETCH = 0,
  ORC_PH_PARTITION,
  ORC_PH_LEAF,
  ORC_PH_HASHPRUNE,
  ORC_PH_ROBUSTPRUNE,
  ORC_PH_SEARCH,
  ORC_PH_BRUTEFORCE,
  ORC_PH_COUNT
};
static double orc_phase_s[ORC_PH_COUNT];

static double orc_now(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}
static void orc_phase_add(int ph, double t0) { orc_phase_s[ph] += orc_now() - t0; }

/* out[ORC_PH_COUNT] receives the summed seconds of sketches, partition, leaf
 * pick, HashPrune, RobustPrune, BeamSearch and brute-force k-NN; returns the
 * count. reset != 0 clears the sums afterwards. */
int orc_phase_seconds(double *out, int reset) {
  for (int i = 0; i < ORC_PH_COUNT; ++i) {
    if (out) out[i] = orc_phase_s[i];
    if (reset) orc_phase_s[i] = 0.0;
  }
  return ORC_PH_COUNT;
}

double orc_dist(const float *a, const float *b, int d, int metric) {
  double s = 0.0;
  if (metric == 0) {
    for (int i = 0; i < d; i++) {
      double t = (double)a[i] - (double)b[i];
      s += t * t;
    }
    return s;
  }
  for (int i = 0; i < d; i++) s += (double)a[i] * (double)b[i];
  return -s;
}

/* ------------------------------------------------------------------ */
/* splitmix64 (Steele, Lea and Flood, 2014): the state advances by the
 * golden-ratio increment and the output is the state passed through the
 * published three-step xor-shift-multiply finaliser. */
static uint64_t sm64_next(uint64_t *state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void orc_splitmix64(uint64_t seed, int64_t count, uint64_t *out) {
  uint64_t s = seed;
  for (int64_t i = 0; i < count; i++) out[i] = sm64_next(&s);
}

/* Key of the child subproblem for bucket t of a subproblem with key `key`. */
static uint64_t child_key(uint64_t key, int64_t t) {
  uint64_t s = key ^ ((uint64_t)(t + 1) * 0x9E3779B97F4A7C15ull);
  return sm64_next(&s);
}

/* floor(r * m / 2^64), the unbiased-enough map of a 64-bit draw to [0, m). */
static uint64_t draw_below(uint64_t r, uint64_t m) {
  return (uint64_t)(((unsigned __int128)r * (unsigned __int128)m) >> 64);
}

/* ------------------------------------------------------------------ */
/* Sketches (Sec. 3, Implementation): Sketch(v)_b = H_b . v, in FP64 with
 * the coordinate index ascending. */
static void orc_sketches_impl(const float *X, int64_t n, int d, const float *H, int m, double *S) {
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < n; p++) {
    for (int b = 0; b < m; b++) {
      double s = 0.0;
      for (int i = 0; i < d; i++) s += (double)H[(int64_t)b * d + i] * (double)X[p * d + i];
      S[p * m + b] = s;
    }
  }
}

/* Residualized hash h_p(c) (Sec. 3, hashing equation): bit b is 1 iff
 * H_b . (c - p) >= 0. With sketches this is Sketch(c)_b >= Sketch(p)_b.
 * Bit 0 is the least significant bit. */
uint16_t orc_hash(const double *sp, const double *sc, int m) {
  uint16_t h = 0;
  for (int b = 0; b < m; b++)
    if (sc[b] >= sp[b]) h |= (uint16_t)(1u << b);
  return h;
}

void orc_hashes(const double *S, int m, const uint32_t *dst, const uint32_t *cand,
                int64_t cnt, uint16_t *out) {
  for (int64_t i = 0; i < cnt; i++)
    out[i] = orc_hash(S + (int64_t)dst[i] * m, S + (int64_t)cand[i] * m, m);
}

/* ------------------------------------------------------------------ */
/* Reservoir distance (Sec. 3, Implementation): stored as bf16. The value is
 * first rounded to float32 (round to nearest even), -0 becomes +0, then the
 * float32 is rounded to bf16 by round-to-nearest-even on the 16 dropped
 * bits. */
uint16_t orc_bf16(double dist) {
  float f = (float)dist;
  if (f == 0.0f) f = 0.0f;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return 0x7FC0; /* NaN */
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}

/* Total order of bf16 values as unsigned 16-bit keys (negative values,
 * possible with the inner-product dissimilarity, sort first). */
static uint32_t bf16_order(uint16_t b) {
  return (b & 0x8000u) ? (uint32_t)(~b & 0xFFFFu) : (uint32_t)(b | 0x8000u);
}

/* Key of a reservoir entry: (bf16 distance, point id), compared
 * lexicographically. A total order is needed for the history-independence
 * theorem of Sec. 3 to hold when distances tie. */
static uint64_t entry_key(uint16_t bf, uint32_t id) {
  return ((uint64_t)bf16_order(bf) << 32) | (uint64_t)id;
}

static uint64_t slot_pack(uint32_t id, uint16_t hash, uint16_t bf) {
  return (uint64_t)id | ((uint64_t)hash << 32) | ((uint64_t)bf << 48);
}
static uint32_t slot_id(uint64_t s) { return (uint32_t)(s & 0xFFFFFFFFu); }
static uint16_t slot_hash(uint64_t s) { return (uint16_t)((s >> 32) & 0xFFFFu); }
static uint16_t slot_bf(uint64_t s) { return (uint16_t)(s >> 48); }

uint64_t orc_empty_slot(void) { return slot_pack(ORC_EMPTY_ID, 0, ORC_BF16_INF); }

void orc_reservoir_init(uint64_t *res, int64_t n, int l_max) {
  uint64_t e = orc_empty_slot();
  for (int64_t i = 0; i < n * (int64_t)l_max; i++) res[i] = e;
}

static int cmp_slot_key(const void *a, const void *b) {
  uint64_t sa = *(const uint64_t *)a, sb = *(const uint64_t *)b;
  int ea = slot_id(sa) == ORC_EMPTY_ID, eb = slot_id(sb) == ORC_EMPTY_ID;
  if (ea != eb) return ea - eb;
  uint64_t ka = entry_key(slot_bf(sa), slot_id(sa));
  uint64_t kb = entry_key(slot_bf(sb), slot_id(sb));
  return (ka > kb) - (ka < kb);
}

/* Canonical reservoir layout: valid slots sorted by (bf16 distance, id),
 * empty slots last. */
void orc_reservoir_canonical(const uint64_t *in, uint64_t *out, int64_t n, int l_max) {
  if (out != in) memcpy(out, in, sizeof(uint64_t) * (size_t)n * (size_t)l_max);
  uint64_t e = orc_empty_slot();
  for (int64_t p = 0; p < n; p++) {
    uint64_t *r = out + p * l_max;
    for (int i = 0; i < l_max; i++)
      if (slot_id(r[i]) == ORC_EMPTY_ID) r[i] = e;
    qsort(r, (size_t)l_max, sizeof(uint64_t), cmp_slot_key);
  }
}

/* Stable grouping of record indices by destination (counting sort). */
static int64_t *group_by_dst(const uint32_t *dst, int64_t cnt, int64_t n, int64_t **order_out) {
  int64_t *start = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t i = 0; i < cnt; i++) start[dst[i] + 1]++;
  for (int64_t p = 0; p < n; p++) start[p + 1] += start[p];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  memcpy(fill, start, sizeof(int64_t) * (size_t)(n + 1));
  int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cnt > 0 ? cnt : 1));
  for (int64_t i = 0; i < cnt; i++) order[fill[dst[i]]++] = i;
  free(fill);
  *order_out = order;
  return start;
}

static int check_ids(const uint32_t *dst, const uint32_t *cand, int64_t cnt, int64_t n) {
  for (int64_t i = 0; i < cnt; i++)
    if ((int64_t)dst[i] >= n || (int64_t)cand[i] >= n) return -1;
  return 0;
}

/* HashPrune, streaming form (Alg. 3), for every destination p, consuming
 * the records addressed to p in the order given. The existing reservoir is
 * the initial key-value store M. Every comparison of distances is a
 * comparison of keys (bf16 distance, id):
 *   - if M holds the bucket h_p(c): keep the smaller key (collision branch);
 *   - else if |M| < l_max: insert c;
 *   - else: let z be the largest key in M; if key(c) < key(z), evict z and
 *     insert c.
 * Records with dst == cand are ignored. Returns -1 on an id >= n. */
static int orc_hashprune_stream_impl(uint64_t *res, int64_t n, int l_max, const double *S, int m,
                         const uint32_t *dst, const uint32_t *cand, const double *dist,
                         int64_t cnt) {
  if (check_ids(dst, cand, cnt, n)) return -1;
  int64_t *order;
  int64_t *start = group_by_dst(dst, cnt, n, &order);
#pragma omp parallel
  {
    uint32_t *mid = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)l_max);
    uint16_t *mh = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)l_max);
    uint16_t *mb = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)l_max);
#pragma omp for schedule(dynamic, 256)
    for (int64_t p = 0; p < n; p++) {
      uint64_t *r = res + p * l_max;
      int sz = 0;
      for (int i = 0; i < l_max; i++) {
        if (slot_id(r[i]) == ORC_EMPTY_ID) continue;
        mid[sz] = slot_id(r[i]);
        mh[sz] = slot_hash(r[i]);
        mb[sz] = slot_bf(r[i]);
        sz++;
      }
      for (int64_t q = start[p]; q < start[p + 1]; q++) {
        int64_t ri = order[q];
        uint32_t c = cand[ri];
        if (c == (uint32_t)p) continue;
        uint16_t h = orc_hash(S + p * m, S + (int64_t)c * m, m);
        uint16_t bf = orc_bf16(dist[ri]);
        uint64_t kc = entry_key(bf, c);
        int hit = -1;
        for (int i = 0; i < sz; i++)
          if (mh[i] == h) { hit = i; break; }
        if (hit >= 0) {
          if (kc < entry_key(mb[hit], mid[hit])) { mid[hit] = c; mb[hit] = bf; }
        } else if (sz < l_max) {
          mid[sz] = c; mh[sz] = h; mb[sz] = bf; sz++;
        } else {
          int z = 0;
          for (int i = 1; i < sz; i++)
            if (entry_key(mb[i], mid[i]) > entry_key(mb[z], mid[z])) z = i;
          if (kc < entry_key(mb[z], mid[z])) { mid[z] = c; mh[z] = h; mb[z] = bf; }
        }
      }
      for (int i = 0; i < l_max; i++)
        r[i] = i < sz ? slot_pack(mid[i], mh[i], mb[i]) : orc_empty_slot();
      qsort(r, (size_t)l_max, sizeof(uint64_t), cmp_slot_key);
    }
    free(mid); free(mh); free(mb);
  }
  free(start);
  free(order);
  return 0;
}

typedef struct { uint64_t key; uint32_t id; uint16_t hash; uint16_t bf; } orc_entry;

static int cmp_entry_hash_key(const void *a, const void *b) {
  const orc_entry *x = (const orc_entry *)a, *y = (const orc_entry *)b;
  if (x->hash != y->hash) return x->hash < y->hash ? -1 : 1;
  return (x->key > y->key) - (x->key < y->key);
}
static int cmp_entry_key(const void *a, const void *b) {
  const orc_entry *x = (const orc_entry *)a, *y = (const orc_entry *)b;
  return (x->key > y->key) - (x->key < y->key);
}

/* HashPrune, closed form (Supplement, history-independence lemma): the
 * reservoir of p ends up holding the l_max smallest keys among the
 * minimum-key entry of every hash bucket, taken over the existing
 * reservoir and all records addressed to p. */
static int orc_hashprune_closed_impl(uint64_t *res, int64_t n, int l_max, const double *S, int m,
                         const uint32_t *dst, const uint32_t *cand, const double *dist,
                         int64_t cnt) {
  if (check_ids(dst, cand, cnt, n)) return -1;
  int64_t *order;
  int64_t *start = group_by_dst(dst, cnt, n, &order);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t p = 0; p < n; p++) {
    uint64_t *r = res + p * l_max;
    int64_t tot = l_max + (start[p + 1] - start[p]);
    orc_entry *e = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)tot);
    int64_t ne = 0;
    for (int i = 0; i < l_max; i++) {
      if (slot_id(r[i]) == ORC_EMPTY_ID) continue;
      e[ne].id = slot_id(r[i]); e[ne].hash = slot_hash(r[i]); e[ne].bf = slot_bf(r[i]);
      e[ne].key = entry_key(e[ne].bf, e[ne].id);
      ne++;
    }
    for (int64_t q = start[p]; q < start[p + 1]; q++) {
      int64_t ri = order[q];
      uint32_t c = cand[ri];
      if (c == (uint32_t)p) continue;
      e[ne].id = c;
      e[ne].hash = orc_hash(S + p * m, S + (int64_t)c * m, m);
      e[ne].bf = orc_bf16(dist[ri]);
      e[ne].key = entry_key(e[ne].bf, c);
      ne++;
    }
    /* per-bucket minimum */
    qsort(e, (size_t)ne, sizeof(orc_entry), cmp_entry_hash_key);
    int64_t nb = 0;
    for (int64_t i = 0; i < ne; i++)
      if (i == 0 || e[i].hash != e[i - 1].hash) e[nb++] = e[i];
    /* l_max smallest bucket minima */
    qsort(e, (size_t)nb, sizeof(orc_entry), cmp_entry_key);
    for (int i = 0; i < l_max; i++)
      r[i] = i < nb ? slot_pack(e[i].id, e[i].hash, e[i].bf) : orc_empty_slot();
    free(e);
  }
  free(start);
  free(order);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Randomized Ball Carving with fanout (Alg. 5, Sec. 4.1).
 *
 * Readings of what the paper leaves open:
 *  - leader count: l = min(leader_cap, max(2, ceil(|P| / leader_div)), |P|)
 *    (P_samp = 1/leader_div, with the hard cap of Sec. 4.1);
 *  - SampleLeaders: the first l entries of a partial Fisher-Yates shuffle of
 *    P in ascending id order, drawing j = t + floor(r * (|P| - t) / 2^64)
 *    from a splitmix64 stream whose state starts at the subproblem key (the
 *    root key is the seed);
 *  - local fanout f = min(fanout[min(depth, 3)], l): each x joins the
 *    buckets of its f nearest leaders by (distance, leader index t);
 *  - Merge: buckets with 0 < |b| < C_min, taken in increasing t, are
 *    grouped greedily, a new group starting when the running sum of bucket
 *    sizes would exceed C_max; each group becomes one leaf holding the union
 *    of its buckets (duplicates removed, ascending);
 *  - buckets with |b| > C_max recurse with the child key of (key, t); a
 *    bucket equal to its whole parent (no progress) is instead cut into
 *    ceil(|P| / C_max) near-equal runs of ascending ids;
 *  - every other bucket is a leaf. Members of a leaf are ascending ids.
 */
typedef struct {
  int64_t *off;
  int64_t n_leaves, cap_leaves;
  uint32_t *mem;
  int64_t n_mem, cap_mem;
  int64_t leader_dists;
} leafbuf;

static void emit_leaf(leafbuf *lb, const uint32_t *ids, int64_t cnt) {
  if (lb->n_leaves + 1 < lb->cap_leaves) lb->off[lb->n_leaves + 1] = lb->n_mem + cnt;
  if (lb->n_mem + cnt <= lb->cap_mem) memcpy(lb->mem + lb->n_mem, ids, sizeof(uint32_t) * (size_t)cnt);
  lb->n_leaves++;
  lb->n_mem += cnt;
}

static int cmp_u32(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  return (x > y) - (x < y);
}

static void rbc(const float *X, int d, const orc_params *prm, const uint32_t *P, int64_t np,
                int depth, uint64_t key, leafbuf *lb) {
  if (np <= prm->c_max) {
    emit_leaf(lb, P, np);
    return;
  }
  int64_t ell = (np + prm->leader_div - 1) / prm->leader_div;
  if (ell < 2) ell = 2;
  if (ell > prm->leader_cap) ell = prm->leader_cap;
  if (ell > np) ell = np;

  /* SampleLeaders */
  uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)np);
  for (int64_t i = 0; i < np; i++) perm[i] = (uint32_t)i;
  uint64_t st = key;
  uint32_t *leaders = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)ell);
  for (int64_t t = 0; t < ell; t++) {
    uint64_t r = sm64_next(&st);
    int64_t j = t + (int64_t)draw_below(r, (uint64_t)(np - t));
    uint32_t tmp = perm[t]; perm[t] = perm[j]; perm[j] = tmp;
    leaders[t] = P[perm[t]];
  }
  free(perm);

  int dd = depth < 3 ? depth : 3;
  int64_t f = prm->fanout[dd];
  if (f > ell) f = ell;
  if (f < 1) f = 1;

  /* each x joins its f nearest leaders by (distance, t) */
  int32_t *asg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(np * f));
#pragma omp parallel
  {
    double *bd = (double *)malloc(sizeof(double) * (size_t)f);
#pragma omp for schedule(static)
    for (int64_t x = 0; x < np; x++) {
      int32_t *bt = asg + x * f;
      int64_t cnt = 0;
      const float *xv = X + (int64_t)P[x] * d;
      for (int64_t t = 0; t < ell; t++) {
        double dv = orc_dist(xv, X + (int64_t)leaders[t] * d, d, prm->metric);
        /* insertion into the sorted list of the f best (ties: smaller t first,
           which holds because t is visited in increasing order and a strict
           comparison is used) */
        if (cnt == f && !(dv < bd[f - 1])) continue;
        int64_t pos = cnt < f ? cnt : f - 1;
        while (pos > 0 && dv < bd[pos - 1]) {
          bd[pos] = bd[pos - 1];
          bt[pos] = bt[pos - 1];
          pos--;
        }
        bd[pos] = dv;
        bt[pos] = (int32_t)t;
        if (cnt < f) cnt++;
      }
    }
    free(bd);
  }
  free(leaders);
  lb->leader_dists += np * ell;

  /* buckets, each in ascending id order */
  int64_t *bstart = (int64_t *)calloc((size_t)ell + 1, sizeof(int64_t));
  for (int64_t i = 0; i < np * f; i++) bstart[asg[i] + 1]++;
  for (int64_t t = 0; t < ell; t++) bstart[t + 1] += bstart[t];
  int64_t *bfill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ell + 1));
  memcpy(bfill, bstart, sizeof(int64_t) * (size_t)(ell + 1));
  uint32_t *bmem = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(np * f));
  for (int64_t x = 0; x < np; x++)
    for (int64_t s = 0; s < f; s++) bmem[bfill[asg[x * f + s]]++] = P[x];
  free(bfill);
  free(asg);

  /* Merge small buckets */
  uint32_t *grp = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(prm->c_max > 0 ? prm->c_max : 1));
  int64_t gsum = 0, gcnt = 0;
  for (int64_t t = 0; t < ell; t++) {
    int64_t sz = bstart[t + 1] - bstart[t];
    if (sz == 0 || sz >= prm->c_min) continue;
    if (gcnt > 0 && gsum + sz > prm->c_max) {
      qsort(grp, (size_t)gsum, sizeof(uint32_t), cmp_u32);
      int64_t u = 0;
      for (int64_t i = 0; i < gsum; i++)
        if (i == 0 || grp[i] != grp[i - 1]) grp[u++] = grp[i];
      emit_leaf(lb, grp, u);
      gsum = 0;
      gcnt = 0;
    }
    memcpy(grp + gsum, bmem + bstart[t], sizeof(uint32_t) * (size_t)sz);
    gsum += sz;
    gcnt++;
  }
  if (gcnt > 0) {
    qsort(grp, (size_t)gsum, sizeof(uint32_t), cmp_u32);
    int64_t u = 0;
    for (int64_t i = 0; i < gsum; i++)
      if (i == 0 || grp[i] != grp[i - 1]) grp[u++] = grp[i];
    emit_leaf(lb, grp, u);
  }
  free(grp);

  /* remaining buckets: leaves, chunked runs, or recursion */
  for (int64_t t = 0; t < ell; t++) {
    int64_t sz = bstart[t + 1] - bstart[t];
    if (sz == 0 || sz < prm->c_min) continue;
    const uint32_t *b = bmem + bstart[t];
    if (sz <= prm->c_max) {
      emit_leaf(lb, b, sz);
    } else if (sz == np) {
      int64_t q = (np + prm->c_max - 1) / prm->c_max;
      int64_t base = np / q, extra = np % q, pos = 0;
      for (int64_t c = 0; c < q; c++) {
        int64_t len = base + (c < extra ? 1 : 0);
        emit_leaf(lb, b + pos, len);
        pos += len;
      }
    } else {
      rbc(X, d, prm, b, sz, depth + 1, child_key(key, t), lb);
    }
  }
  free(bmem);
  free(bstart);
}

/* Partition all n points. Leaves are written as CSR (offsets[n_leaves+1],
 * members). Returns 0, or -1 if a capacity was too small (the needed sizes
 * are still written to *n_leaves_out and *n_members_out). */
static int orc_partition_impl(const float *X, int64_t n, int d, const orc_params *prm, int64_t *offsets,
                  int64_t cap_leaves, uint32_t *members, int64_t cap_members,
                  int64_t *n_leaves_out, int64_t *n_members_out, int64_t *leader_dists_out) {
  leafbuf lb;
  lb.off = offsets;
  lb.cap_leaves = cap_leaves + 1;
  lb.n_leaves = 0;
  lb.mem = members;
  lb.cap_mem = cap_members;
  lb.n_mem = 0;
  lb.leader_dists = 0;
  if (cap_leaves >= 0) offsets[0] = 0;
  uint32_t *P = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
  for (int64_t i = 0; i < n; i++) P[i] = (uint32_t)i;
  rbc(X, d, prm, P, n, 0, prm->seed, &lb);
  free(P);
  *n_leaves_out = lb.n_leaves;
  *n_members_out = lb.n_mem;
  if (leader_dists_out) *leader_dists_out = lb.leader_dists;
  return (lb.n_leaves > cap_leaves || lb.n_mem > cap_members) ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Low-precision GEMM operands (precision forms of the leaf GEMM).
 * The paper computes leaf distances in full precision; a reduced-precision
 * leaf GEMM is this library's extension. Its operand encodings follow the
 * published format definitions:
 *   bf16: the upper 16 bits of IEEE binary32 after round-to-nearest-even;
 *   fp16: IEEE 754 binary16 (5 exponent bits, bias 15, 10 fraction bits,
 *         subnormals), round-to-nearest-even, overflow to infinity;
 *   fp8:  OCP 8-bit floating point, E4M3 ("e4m3fn": bias 7, 3 fraction
 *         bits, subnormals, no infinities, S.1111.111 = NaN, largest finite
 *         448), round-to-nearest-even, saturating at +-448. Each point is
 *         scaled by s = 448 / max_i |x_i| (computed in binary32; s = 1 for a
 *         zero vector) before encoding, and decodes as code * (max / 448).  */
#define ORC_PREC_FP32 0
#define ORC_PREC_BF16 1
#define ORC_PREC_FP8 2
#define ORC_PREC_FP16 3

static uint32_t f32_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}

uint16_t orc_bf16_rne(float f) {
  uint32_t u = f32_bits(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

double orc_bf16_value(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return (double)f;
}

/* Round a non-negative finite double that is a binary32 value to an
 * integer, ties to even. */
static double rne_int(double v) {
  double fl = floor(v), fr = v - fl;
  if (fr > 0.5) return fl + 1.0;
  if (fr < 0.5) return fl;
  return fmod(fl, 2.0) == 0.0 ? fl : fl + 1.0;
}

uint16_t orc_fp16_rne(float f) {
  uint32_t u = f32_bits(f);
  uint16_t sign = (uint16_t)((u >> 16) & 0x8000u);
  double a = fabs((double)f);
  if (isnan(a)) return (uint16_t)(sign | 0x7E00u);
  /* the largest finite binary16 is 65504; halfway to the next step (65536)
   * is 65520, which rounds (to even) up to infinity */
  if (a >= 65520.0) return (uint16_t)(sign | 0x7C00u);
  if (a < ldexp(1.0, -14)) {
    /* subnormal: value = m * 2^-24, m in 0..1024 (1024 is the smallest normal) */
    double m = rne_int(a * ldexp(1.0, 24));
    return (uint16_t)(sign | (uint16_t)m);
  }
  int e;
  double fr = frexp(a, &e); /* a = fr * 2^e, fr in [0.5, 1) */
  int E = e - 1;            /* a = (2 fr) * 2^E, 2 fr in [1, 2) */
  double m = rne_int((2.0 * fr - 1.0) * 1024.0);
  if (m == 1024.0) {
    m = 0.0;
    E += 1;
  }
  return (uint16_t)(sign | (uint16_t)((E + 15) << 10) | (uint16_t)m);
}

double orc_fp16_value(uint16_t h) {
  int s = (h >> 15) & 1, e = (h >> 10) & 31, m = h & 1023;
  double v;
  if (e == 31) v = m ? NAN : INFINITY;
  else if (e == 0) v = ldexp((double)m, -24);
  else v = ldexp(1.0 + m / 1024.0, e - 15);
  return s ? -v : v;
}

uint8_t orc_e4m3_rne_sat(float f) {
  uint8_t sign = (f32_bits(f) >> 24) & 0x80u;
  double a = fabs((double)f);
  if (isnan(a)) return (uint8_t)(sign | 0x7Fu);
  if (a >= 448.0) return (uint8_t)(sign | 0x7Eu); /* saturate to the largest finite */
  if (a < ldexp(1.0, -6)) {
    /* subnormal: value = m * 2^-9, m in 0..8 (8 is the smallest normal, code 0x08) */
    double m = rne_int(a * 512.0);
    return (uint8_t)(sign | (uint8_t)m);
  }
  int e;
  double fr = frexp(a, &e);
  int E = e - 1;
  double m = rne_int((2.0 * fr - 1.0) * 8.0);
  if (m == 8.0) {
    m = 0.0;
    E += 1;
  }
  /* 448 <= value would need E = 8, m = 7 (the NaN pattern); unreachable
   * here because a < 448 and the largest finite value is 448 (E 8, m 6) */
  return (uint8_t)(sign | (uint8_t)((E + 7) << 3) | (uint8_t)m);
}

double orc_e4m3_value(uint8_t c) {
  int s = (c >> 7) & 1, e = (c >> 3) & 15, m = c & 7;
  double v;
  if (e == 15 && m == 7) v = NAN;
  else if (e == 0) v = ldexp((double)m, -9);
  else v = ldexp(1.0 + m / 8.0, e - 7);
  return s ? -v : v;
}

/* Quantize the rows of X (n x d) to a GEMM operand. codes: n x d uint16
 * (bf16, fp16) or uint8 (fp8); inv_scale: n floats (fp8: max_i |x_i| / 448
 * in binary32, or 1 for a zero row; other precisions: 1); xq: the decoded
 * operand in FP64 (n x d), code value times inv_scale. prec FP32 copies X. */
void orc_quantize(const float *X, int64_t n, int d, int prec, void *codes, float *inv_scale,
                  double *xq) {
  for (int64_t p = 0; p < n; p++) {
    const float *x = X + p * d;
    float inv = 1.0f, s = 1.0f;
    if (prec == ORC_PREC_FP8) {
      float mx = 0.0f;
      for (int i = 0; i < d; i++) {
        float a = fabsf(x[i]);
        if (a > mx) mx = a;
      }
      if (mx > 0.0f) {
        s = 448.0f / mx;
        inv = mx / 448.0f;
      }
    }
    if (inv_scale) inv_scale[p] = inv;
    for (int i = 0; i < d; i++) {
      double v;
      if (prec == ORC_PREC_BF16) {
        uint16_t c = orc_bf16_rne(x[i]);
        if (codes) ((uint16_t *)codes)[p * d + i] = c;
        v = orc_bf16_value(c);
      } else if (prec == ORC_PREC_FP16) {
        uint16_t c = orc_fp16_rne(x[i]);
        if (codes) ((uint16_t *)codes)[p * d + i] = c;
        v = orc_fp16_value(c);
      } else if (prec == ORC_PREC_FP8) {
        float t = x[i] * s; /* binary32 product, as the encoder sees it */
        uint8_t c = orc_e4m3_rne_sat(t);
        if (codes) ((uint8_t *)codes)[p * d + i] = c;
        v = orc_e4m3_value(c) * (double)inv;
      } else {
        if (codes) ((float *)codes)[p * d + i] = x[i];
        v = (double)x[i];
      }
      if (xq) xq[p * d + i] = v;
    }
  }
}

static double dist64(const double *a, const double *b, int d, int metric) {
  double s = 0.0;
  if (metric == 0) {
    for (int i = 0; i < d; i++) {
      double t = a[i] - b[i];
      s += t * t;
    }
    return s;
  }
  for (int i = 0; i < d; i++) s += a[i] * b[i];
  return -s;
}

/* Leaf pick with a reduced-precision GEMM distance and rescoring, in the
 * independent (FP64) mode. For every member i of a leaf: the k1 nearest
 * co-members j != i by (distance between the decoded operands xq_i, xq_j,
 * id_j) -- the value a low-precision GEMM approximates -- then those k1
 * re-ranked by (distance between the original vectors, id) and the first k
 * kept. k1 = mult * k, or k + extra when mult = 0; with both 0 the k nearest
 * by the operand distance are kept without re-ranking. Emitted distances
 * are always those of the original vectors. Output layout as orc_leaf_knn. */
static void orc_leaf_knn_lowp_impl(const float *X, const double *xq, int d, int metric,
                       const int64_t *offsets, const uint32_t *members, int64_t n_leaves, int k,
                       int mult, int extra, uint32_t *out_cand, double *out_dist) {
  const int k1 = mult > 0 ? mult * k : k + extra;
  const int rerank = mult > 0 || extra > 0;
#pragma omp parallel
  {
    double *bd = (double *)malloc(sizeof(double) * (size_t)k1);
    uint32_t *bi = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)k1);
    double *rd = (double *)malloc(sizeof(double) * (size_t)k1);
#pragma omp for schedule(dynamic, 1)
    for (int64_t L = 0; L < n_leaves; L++) {
      int64_t o = offsets[L], s = offsets[L + 1] - offsets[L];
      for (int64_t i = 0; i < s; i++) {
        uint32_t pi = members[o + i];
        int cnt = 0;
        for (int64_t j = 0; j < s; j++) {
          if (j == i) continue;
          uint32_t pj = members[o + j];
          double dv = dist64(xq + (int64_t)pi * d, xq + (int64_t)pj * d, d, metric);
          if (cnt == k1 && !(dv < bd[k1 - 1] || (dv == bd[k1 - 1] && pj < bi[k1 - 1]))) continue;
          int pos = cnt < k1 ? cnt : k1 - 1;
          while (pos > 0 && (dv < bd[pos - 1] || (dv == bd[pos - 1] && pj < bi[pos - 1]))) {
            bd[pos] = bd[pos - 1];
            bi[pos] = bi[pos - 1];
            pos--;
          }
          bd[pos] = dv;
          bi[pos] = pj;
          if (cnt < k1) cnt++;
        }
        /* distances of the original vectors; re-rank when rescoring */
        for (int r = 0; r < cnt; r++)
          rd[r] = orc_dist(X + (int64_t)pi * d, X + (int64_t)bi[r] * d, d, metric);
        if (rerank) {
          for (int a = 1; a < cnt; a++) {
            double dv = rd[a];
            uint32_t iv = bi[a];
            int b = a;
            while (b > 0 && (rd[b - 1] > dv || (rd[b - 1] == dv && bi[b - 1] > iv))) {
              rd[b] = rd[b - 1];
              bi[b] = bi[b - 1];
              b--;
            }
            rd[b] = dv;
            bi[b] = iv;
          }
          if (cnt > k) cnt = k;
        }
        for (int r = 0; r < k; r++) {
          out_cand[(o + i) * k + r] = r < cnt ? bi[r] : ORC_EMPTY_ID;
          out_dist[(o + i) * k + r] = r < cnt ? rd[r] : INFINITY;
        }
      }
    }
    free(bd);
    free(bi);
    free(rd);
  }
}

/* ------------------------------------------------------------------ */
/* Leaf pick (Sec. 4.2): for every member i of a leaf, its k' = min(k, s-1)
 * nearest co-members j != i by (distance, id). Output rows follow the CSR
 * member order: row r = offsets[leaf] + i holds k slots; unused slots have
 * cand = 0xFFFFFFFF. The bi-directed records are (dst=i, cand=j, d) and
 * (dst=j, cand=i, d). */
static void orc_leaf_knn_impl(const float *X, int d, int metric, const int64_t *offsets,
                  const uint32_t *members, int64_t n_leaves, int k, uint32_t *out_cand,
                  double *out_dist) {
#pragma omp parallel
  {
    double *bd = (double *)malloc(sizeof(double) * (size_t)k);
    uint32_t *bi = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)k);
#pragma omp for schedule(dynamic, 1)
    for (int64_t L = 0; L < n_leaves; L++) {
      int64_t o = offsets[L], s = offsets[L + 1] - offsets[L];
      for (int64_t i = 0; i < s; i++) {
        uint32_t pi = members[o + i];
        int cnt = 0;
        for (int64_t j = 0; j < s; j++) {
          if (j == i) continue;
          uint32_t pj = members[o + j];
          double dv = orc_dist(X + (int64_t)pi * d, X + (int64_t)pj * d, d, metric);
          if (cnt == k && !(dv < bd[k - 1] || (dv == bd[k - 1] && pj < bi[k - 1]))) continue;
          int pos = cnt < k ? cnt : k - 1;
          while (pos > 0 && (dv < bd[pos - 1] || (dv == bd[pos - 1] && pj < bi[pos - 1]))) {
            bd[pos] = bd[pos - 1];
            bi[pos] = bi[pos - 1];
            pos--;
          }
          bd[pos] = dv;
          bi[pos] = pj;
          if (cnt < k) cnt++;
        }
        for (int r = 0; r < k; r++) {
          out_cand[(o + i) * k + r] = r < cnt ? bi[r] : ORC_EMPTY_ID;
          out_dist[(o + i) * k + r] = r < cnt ? bd[r] : INFINITY;
        }
      }
    }
    free(bd);
    free(bi);
  }
}

/* Per-row selection from a given float32 matrix (replay of distances
 * computed elsewhere): the k smallest (D[r][c], c) with c != self_col[r]
 * (self_col may be NULL or hold -1). Unused slots get 0xFFFFFFFF. */
void orc_topk_rows(const float *D, int64_t rows, int64_t cols, int k, const int64_t *self_col,
                   uint32_t *out_col, float *out_val) {
#pragma omp parallel
  {
    float *bd = (float *)malloc(sizeof(float) * (size_t)k);
    uint32_t *bi = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)k);
#pragma omp for schedule(static)
    for (int64_t r = 0; r < rows; r++) {
      int cnt = 0;
      int64_t sc = self_col ? self_col[r] : -1;
      for (int64_t c = 0; c < cols; c++) {
        if (c == sc) continue;
        float v = D[r * cols + c];
        if (cnt == k && !(v < bd[k - 1])) continue;
        int pos = cnt < k ? cnt : k - 1;
        while (pos > 0 && v < bd[pos - 1]) {
          bd[pos] = bd[pos - 1];
          bi[pos] = bi[pos - 1];
          pos--;
        }
        bd[pos] = v;
        bi[pos] = (uint32_t)c;
        if (cnt < k) cnt++;
      }
      for (int i = 0; i < k; i++) {
        out_col[r * k + i] = i < cnt ? bi[i] : ORC_EMPTY_ID;
        if (out_val) out_val[r * k + i] = i < cnt ? bd[i] : INFINITY;
      }
    }
    free(bd);
    free(bi);
  }
}

/* ------------------------------------------------------------------ */
/* RobustPrune (Alg. 2) on the reservoir of every point x.
 * The candidate set N is the reservoir's ids, with d(x, c) recomputed in
 * FP64; "argmin" is over N by (distance, id). alpha is the float32 value
 * widened to FP64; a candidate z is removed when alpha * d(y, z) < d(x, z)
 * (strict). The output holds at most R ids in admission order, padded with
 * 0xFFFFFFFF.
 *  lazy = 0: the standard loop of Alg. 2.
 *  lazy = 1: the lazy form (Supplement, "Optimizing RobustPrune"): walk the
 *            candidates in (distance, id) order and admit c unless an
 *            already-admitted y prunes it.                                    */
typedef struct { double d; uint32_t id; } dcand;
static int cmp_dcand(const void *a, const void *b) {
  const dcand *x = (const dcand *)a, *y = (const dcand *)b;
  if (x->d != y->d) return x->d < y->d ? -1 : 1;
  return (x->id > y->id) - (x->id < y->id);
}

static void orc_robustprune_impl(const float *X, int d, int metric, const uint64_t *res, int64_t n,
                     int l_max, float alpha_f, int R, int lazy, uint32_t *graph,
                     uint32_t *degree) {
  double alpha = (double)alpha_f;
#pragma omp parallel
  {
    dcand *N = (dcand *)malloc(sizeof(dcand) * (size_t)l_max);
    char *alive = (char *)malloc((size_t)l_max);
    uint32_t *E = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(R > 0 ? R : 1));
#pragma omp for schedule(dynamic, 64)
    for (int64_t x = 0; x < n; x++) {
      const float *xv = X + x * d;
      int nn = 0;
      for (int i = 0; i < l_max; i++) {
        uint32_t c = slot_id(res[x * l_max + i]);
        if (c == ORC_EMPTY_ID || (int64_t)c == x) continue;
        N[nn].id = c;
        N[nn].d = orc_dist(xv, X + (int64_t)c * d, d, metric);
        nn++;
      }
      int ne = 0;
      if (!lazy) {
        for (int i = 0; i < nn; i++) alive[i] = 1;
        for (;;) {
          if (ne >= R) break;
          int best = -1;
          for (int i = 0; i < nn; i++) {
            if (!alive[i]) continue;
            if (best < 0 || N[i].d < N[best].d || (N[i].d == N[best].d && N[i].id < N[best].id))
              best = i;
          }
          if (best < 0) break;
          uint32_t y = N[best].id;
          E[ne++] = y;
          alive[best] = 0;
          const float *yv = X + (int64_t)y * d;
          for (int i = 0; i < nn; i++) {
            if (!alive[i]) continue;
            double dyz = orc_dist(yv, X + (int64_t)N[i].id * d, d, metric);
            if (alpha * dyz < N[i].d) alive[i] = 0;
          }
        }
      } else {
        qsort(N, (size_t)nn, sizeof(dcand), cmp_dcand);
        for (int i = 0; i < nn && ne < R; i++) {
          const float *cv = X + (int64_t)N[i].id * d;
          int pruned = 0;
          for (int e = 0; e < ne && !pruned; e++) {
            double dyc = orc_dist(X + (int64_t)E[e] * d, cv, d, metric);
            if (alpha * dyc < N[i].d) pruned = 1;
          }
          if (!pruned) E[ne++] = N[i].id;
        }
      }
      for (int i = 0; i < R; i++) graph[x * R + i] = i < ne ? E[i] : ORC_EMPTY_ID;
      degree[x] = (uint32_t)ne;
    }
    free(N);
    free(alive);
    free(E);
  }
}

/* ------------------------------------------------------------------ */
/* BeamSearch (Alg. 1). The beam B holds at most L entries ordered by
 * (distance to q, id); a `seen` set stops a point from entering the beam
 * twice. Each step visits the closest unvisited beam entry, inserts its
 * unseen neighbours, and truncates B to L. It stops when every beam entry
 * is visited and returns the first k entries. cmps counts evaluations of
 * d(q, .), the start included. */
/* Lazy RobustPrune (as in orc_robustprune) of the listed points only:
 * point xs[i] uses reservoir row res[i] and writes graph row i. */
static void orc_robustprune_points_impl(const float *X, int d, int metric, const uint64_t *res,
                            const uint32_t *xs, int64_t nx, int l_max, float alpha_f, int R,
                            uint32_t *graph, uint32_t *degree) {
  double alpha = (double)alpha_f;
#pragma omp parallel
  {
    dcand *N = (dcand *)malloc(sizeof(dcand) * (size_t)l_max);
    uint32_t *E = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(R > 0 ? R : 1));
#pragma omp for schedule(dynamic, 16)
    for (int64_t i0 = 0; i0 < nx; i0++) {
      const uint32_t x = xs[i0];
      const float *xv = X + (int64_t)x * d;
      int nn = 0;
      for (int i = 0; i < l_max; i++) {
        uint32_t c = slot_id(res[i0 * l_max + i]);
        if (c == ORC_EMPTY_ID || c == x) continue;
        N[nn].id = c;
        N[nn].d = orc_dist(xv, X + (int64_t)c * d, d, metric);
        nn++;
      }
      qsort(N, (size_t)nn, sizeof(dcand), cmp_dcand);
      int ne = 0;
      for (int i = 0; i < nn && ne < R; i++) {
        const float *cv = X + (int64_t)N[i].id * d;
        int pruned = 0;
        for (int e = 0; e < ne && !pruned; e++) {
          double dyc = orc_dist(X + (int64_t)E[e] * d, cv, d, metric);
          if (alpha * dyc < N[i].d) pruned = 1;
        }
        if (!pruned) E[ne++] = N[i].id;
      }
      for (int i = 0; i < R; i++) graph[i0 * R + i] = i < ne ? E[i] : ORC_EMPTY_ID;
      degree[i0] = (uint32_t)ne;
    }
    free(N);
    free(E);
  }
}

static void orc_beam_search_impl(const float *X, int64_t n, int d, int metric, const uint32_t *graph, int R,
                     const float *Q, int64_t nq, int k, int L, uint32_t start, uint32_t *out_ids,
                     double *out_dist, uint32_t *out_cmps) {
#pragma omp parallel
  {
    dcand *B = (dcand *)malloc(sizeof(dcand) * (size_t)(L + R + 1));
    char *vis = (char *)malloc((size_t)(L + R + 1));
    uint8_t *seen = (uint8_t *)calloc((size_t)(n + 7) / 8, 1);
#pragma omp for schedule(dynamic, 1)
    for (int64_t qi = 0; qi < nq; qi++) {
      const float *qv = Q + qi * d;
      memset(seen, 0, (size_t)(n + 7) / 8);
      int nb = 1;
      B[0].id = start;
      B[0].d = orc_dist(qv, X + (int64_t)start * d, d, metric);
      vis[0] = 0;
      seen[start >> 3] |= (uint8_t)(1u << (start & 7));
      uint32_t cmps = 1;
      for (;;) {
        int cur = -1;
        for (int i = 0; i < nb; i++)
          if (!vis[i]) { cur = i; break; }
        if (cur < 0) break;
        vis[cur] = 1;
        uint32_t p = B[cur].id;
        for (int e = 0; e < R; e++) {
          uint32_t u = graph[(int64_t)p * R + e];
          if (u == ORC_EMPTY_ID) continue;
          if (seen[u >> 3] & (1u << (u & 7))) continue;
          seen[u >> 3] |= (uint8_t)(1u << (u & 7));
          double du = orc_dist(qv, X + (int64_t)u * d, d, metric);
          cmps++;
          /* sorted insertion by (d, id) */
          int pos = nb;
          while (pos > 0 && (du < B[pos - 1].d || (du == B[pos - 1].d && u < B[pos - 1].id))) {
            B[pos] = B[pos - 1];
            vis[pos] = vis[pos - 1];
            pos--;
          }
          B[pos].d = du;
          B[pos].id = u;
          vis[pos] = 0;
          nb++;
        }
        if (nb > L) nb = L;
      }
      for (int i = 0; i < k; i++) {
        out_ids[qi * k + i] = i < nb ? B[i].id : ORC_EMPTY_ID;
        out_dist[qi * k + i] = i < nb ? B[i].d : INFINITY;
      }
      if (out_cmps) out_cmps[qi] = cmps;
    }
    free(B);
    free(vis);
    free(seen);
  }
}

/* Exact k nearest neighbours (Definition of k-NN search), ties by id. */
static void orc_bruteforce_knn_impl(const float *X, int64_t n, int d, int metric, const float *Q, int64_t nq,
                        int k, uint32_t *out_ids, double *out_dist) {
#pragma omp parallel
  {
    double *bd = (double *)malloc(sizeof(double) * (size_t)k);
    uint32_t *bi = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)k);
#pragma omp for schedule(dynamic, 4)
    for (int64_t qi = 0; qi < nq; qi++) {
      int cnt = 0;
      for (int64_t j = 0; j < n; j++) {
        double dv = orc_dist(Q + qi * d, X + j * d, d, metric);
        if (cnt == k && !(dv < bd[k - 1])) continue;
        int pos = cnt < k ? cnt : k - 1;
        while (pos > 0 && dv < bd[pos - 1]) {
          bd[pos] = bd[pos - 1];
          bi[pos] = bi[pos - 1];
          pos--;
        }
        bd[pos] = dv;
        bi[pos] = (uint32_t)j;
        if (cnt < k) cnt++;
      }
      for (int i = 0; i < k; i++) {
        out_ids[qi * k + i] = i < cnt ? bi[i] : ORC_EMPTY_ID;
        out_dist[qi * k + i] = i < cnt ? bd[i] : INFINITY;
      }
    }
    free(bd);
    free(bi);
  }
}

/* Start node for BeamSearch: the point nearest the mean of X by
 * (squared L2 distance, id), in FP64. The paper leaves the source open. */
uint32_t orc_start_node(const float *X, int64_t n, int d, double *dist_out) {
  double *mean = (double *)calloc((size_t)d, sizeof(double));
  for (int64_t p = 0; p < n; p++)
    for (int i = 0; i < d; i++) mean[i] += (double)X[p * d + i];
  for (int i = 0; i < d; i++) mean[i] /= (double)n;
  uint32_t best = 0;
  double bd = INFINITY;
  for (int64_t p = 0; p < n; p++) {
    double s = 0.0;
    for (int i = 0; i < d; i++) {
      double t = (double)X[p * d + i] - mean[i];
      s += t * t;
    }
    if (dist_out) dist_out[p] = s;
    if (s < bd) { bd = s; best = (uint32_t)p; }
  }
  free(mean);
  return best;
}

/* ------------------------------------------------------------------ */
/* Insertion (an extension of this library; the paper builds only). The
 * representative of a leaf is the member m with the smallest
 * (sum_i (s x_mi - S_i)^2, id), S_i the sum of the members' coordinate i
 * (in member order) and s the leaf size: s^2 times the squared distance of
 * m to the leaf mean. Empty leaves get id 0. */
void orc_leaf_reps(const float *X, int d, const int64_t *offsets, const uint32_t *members,
                   int64_t n_leaves, uint32_t *rep) {
#pragma omp parallel
  {
    double *S = (double *)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(dynamic, 1)
    for (int64_t L = 0; L < n_leaves; L++) {
      int64_t o = offsets[L], s = offsets[L + 1] - offsets[L];
      if (s <= 0) {
        rep[L] = 0;
        continue;
      }
      for (int i = 0; i < d; i++) S[i] = 0.0;
      for (int64_t j = 0; j < s; j++)
        for (int i = 0; i < d; i++) S[i] += (double)X[(int64_t)members[o + j] * d + i];
      double best = INFINITY;
      uint32_t bid = 0xFFFFFFFFu;
      for (int64_t j = 0; j < s; j++) {
        uint32_t id = members[o + j];
        double sc = 0.0;
        for (int i = 0; i < d; i++) {
          double t = (double)s * (double)X[(int64_t)id * d + i] - S[i];
          sc += t * t;
        }
        if (sc < best || (sc == best && id < bid)) {
          best = sc;
          bid = id;
        }
      }
      rep[L] = bid;
    }
    free(S);
  }
}

/* ------------------------------------------------------------------ */
/* All-to-All Prune leaf picker (Supplement, "Picking within Leaves",
 * All-to-All Prune): for every member x of a leaf, RobustPrune (Alg. 2, in
 * the lazy form of the Supplement's "Optimizing RobustPrune") with every
 * other member of the leaf as the candidate set N: the candidates are taken
 * in (d(x, c), id) order; c is skipped if an already admitted y has
 * alpha * d(y, c) < d(x, c), else appended; the scan stops once R_leaf are
 * admitted. All distances in FP64. Row i of the CSR (offsets, members)
 * writes out_cand[i * R_leaf ..] (ids in admission order, EMPTY padding)
 * and out_dist (d(x, c) of each, +inf padding). */
static void orc_leaf_all_to_all_impl(const float *X, int d, int metric, const int64_t *offsets,
                                     const uint32_t *members, int64_t n_leaves, int R_leaf,
                                     float alpha_f, uint32_t *out_cand, double *out_dist) {
  const double alpha = (double)alpha_f;
  int64_t max_sz = 0;
  for (int64_t l = 0; l < n_leaves; l++)
    if (offsets[l + 1] - offsets[l] > max_sz) max_sz = offsets[l + 1] - offsets[l];
#pragma omp parallel
  {
    dcand *N = (dcand *)malloc(sizeof(dcand) * (size_t)(max_sz > 0 ? max_sz : 1));
    uint32_t *E = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(R_leaf > 0 ? R_leaf : 1));
    double *ED = (double *)malloc(sizeof(double) * (size_t)(R_leaf > 0 ? R_leaf : 1));
#pragma omp for schedule(dynamic, 1)
    for (int64_t l = 0; l < n_leaves; l++) {
      const int64_t o = offsets[l], sz = offsets[l + 1] - offsets[l];
      for (int64_t i = 0; i < sz; i++) {
        const uint32_t x = members[o + i];
        const float *xv = X + (int64_t)x * d;
        int64_t nn = 0;
        for (int64_t j = 0; j < sz; j++) {
          if (j == i) continue;
          N[nn].id = members[o + j];
          N[nn].d = orc_dist(xv, X + (int64_t)N[nn].id * d, d, metric);
          nn++;
        }
        qsort(N, (size_t)nn, sizeof(dcand), cmp_dcand);
        int ne = 0;
        for (int64_t t = 0; t < nn && ne < R_leaf; t++) {
          const float *cv = X + (int64_t)N[t].id * d;
          int pruned = 0;
          for (int e = 0; e < ne && !pruned; e++)
            if (alpha * orc_dist(X + (int64_t)E[e] * d, cv, d, metric) < N[t].d) pruned = 1;
          if (!pruned) {
            E[ne] = N[t].id;
            ED[ne] = N[t].d;
            ne++;
          }
        }
        for (int e = 0; e < R_leaf; e++) {
          out_cand[(o + i) * R_leaf + e] = e < ne ? E[e] : ORC_EMPTY_ID;
          out_dist[(o + i) * R_leaf + e] = e < ne ? ED[e] : INFINITY;
        }
      }
    }
    free(N);
    free(E);
    free(ED);
  }
}

/* Exported phase functions: the definitions above, timed. */

void orc_sketches(const float *X, int64_t n, int d, const float *H, int m, double *S) {
  const double t0 = orc_now();
  orc_sketches_impl(X, n, d, H, m, S);
  orc_phase_add(ORC_PH_SKETCH, t0);
}

int orc_hashprune_stream(uint64_t *res, int64_t n, int l_max, const double *S, int m, const uint32_t *dst, const uint32_t *cand, const double *dist, int64_t cnt) {
  const double t0 = orc_now();
  const int r = orc_hashprune_stream_impl(res, n, l_max, S, m, dst, cand, dist, cnt);
  orc_phase_add(ORC_PH_HASHPRUNE, t0);
  return r;
}

int orc_hashprune_closed(uint64_t *res, int64_t n, int l_max, const double *S, int m, const uint32_t *dst, const uint32_t *cand, const double *dist, int64_t cnt) {
  const double t0 = orc_now();
  const int r = orc_hashprune_closed_impl(res, n, l_max, S, m, dst, cand, dist, cnt);
  orc_phase_add(ORC_PH_HASHPRUNE, t0);
  return r;
}

int orc_partition(const float *X, int64_t n, int d, const orc_params *prm, int64_t *offsets, int64_t cap_leaves, uint32_t *members, int64_t cap_members, int64_t *n_leaves_out, int64_t *n_members_out, int64_t *leader_dists_out) {
  const double t0 = orc_now();
  const int r = orc_partition_impl(X, n, d, prm, offsets, cap_leaves, members, cap_members, n_leaves_out, n_members_out, leader_dists_out);
  orc_phase_add(ORC_PH_PARTITION, t0);
  return r;
}

void orc_leaf_knn_lowp(const float *X, const double *xq, int d, int metric, const int64_t *offsets, const uint32_t *members, int64_t n_leaves, int k, int mult, int extra, uint32_t *out_cand, double *out_dist) {
  const double t0 = orc_now();
  orc_leaf_knn_lowp_impl(X, xq, d, metric, offsets, members, n_leaves, k, mult, extra, out_cand, out_dist);
  orc_phase_add(ORC_PH_LEAF, t0);
}

void orc_leaf_knn(const float *X, int d, int metric, const int64_t *offsets, const uint32_t *members, int64_t n_leaves, int k, uint32_t *out_cand, double *out_dist) {
  const double t0 = orc_now();
  orc_leaf_knn_impl(X, d, metric, offsets, members, n_leaves, k, out_cand, out_dist);
  orc_phase_add(ORC_PH_LEAF, t0);
}

void orc_robustprune(const float *X, int d, int metric, const uint64_t *res, int64_t n, int l_max, float alpha_f, int R, int lazy, uint32_t *graph, uint32_t *degree) {
  const double t0 = orc_now();
  orc_robustprune_impl(X, d, metric, res, n, l_max, alpha_f, R, lazy, graph, degree);
  orc_phase_add(ORC_PH_ROBUSTPRUNE, t0);
}

void orc_robustprune_points(const float *X, int d, int metric, const uint64_t *res, const uint32_t *xs, int64_t nx, int l_max, float alpha_f, int R, uint32_t *graph, uint32_t *degree) {
  const double t0 = orc_now();
  orc_robustprune_points_impl(X, d, metric, res, xs, nx, l_max, alpha_f, R, graph, degree);
  orc_phase_add(ORC_PH_ROBUSTPRUNE, t0);
}

void orc_beam_search(const float *X, int64_t n, int d, int metric, const uint32_t *graph, int R, const float *Q, int64_t nq, int k, int L, uint32_t start, uint32_t *out_ids, double *out_dist, uint32_t *out_cmps) {
  const double t0 = orc_now();
  orc_beam_search_impl(X, n, d, metric, graph, R, Q, nq, k, L, start, out_ids, out_dist, out_cmps);
  orc_phase_add(ORC_PH_SEARCH, t0);
}

void orc_bruteforce_knn(const float *X, int64_t n, int d, int metric, const float *Q, int64_t nq, int k, uint32_t *out_ids, double *out_dist) {
  const double t0 = orc_now();
  orc_bruteforce_knn_impl(X, n, d, metric, Q, nq, k, out_ids, out_dist);
  orc_phase_add(ORC_PH_BRUTEFORCE, t0);
}

void orc_leaf_all_to_all(const float *X, int d, int metric, const int64_t *offsets,
                         const uint32_t *members, int64_t n_leaves, int R_leaf, float alpha_f,
                         uint32_t *out_cand, double *out_dist) {
  const double t0 = orc_now();
  orc_leaf_all_to_all_impl(X, d, metric, offsets, members, n_leaves, R_leaf, alpha_f, out_cand,
                           out_dist);
  orc_phase_add(ORC_PH_LEAF, t0);
}
