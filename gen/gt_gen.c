/*
 * Seeded synthetic graph generators (CSR with int64 offsets, int32 vertex
 * IDs, optional 32-bit payload words).
 *
 * This module only draws inputs.  It holds none of the transposition's
 * arithmetic: every CSR is produced directly in source order (per-source
 * edge counts first, then each source's list), so no edge list is ever
 * regrouped by key here.
 *
 * Randomness is counter based: every draw is splitmix64 applied to a key
 * made of (graph seed, stream tag, entity, counter), so the output does not
 * depend on the number of OpenMP threads.  splitmix64 follows its published
 * definition (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014; constants as in Vigna's public-domain C code).
 *
 * Families:
 *   R-MAT (Chakrabarti, Zhan, Faloutsos 2004): quadrant probabilities
 *     (a, b, c, d) per level.  Sources are drawn by splitting the edge count
 *     recursively over the source bits (the marginal of a source bit is
 *     c+d for a one); each edge's destination bits are then drawn
 *     conditioned on the source bit of the same level:
 *     P(dst bit = 1 | src bit = 0) = b/(a+b), P(dst bit = 1 | src bit = 1)
 *     = d/(c+d).  Vertices at or above n are excluded (counts are split in
 *     proportion to the admissible mass; destinations >= n are redrawn).
 *     Binomial splits use exact inversion up to 1000 trials and a rounded
 *     normal approximation above that.
 *   uniform: out-degree exactly ef per vertex, destinations iid uniform.
 *   geometric locality: dst = (src + o) mod n, o = 1 + floor(ln U / ln(1-p)).
 * Optional ID permutation: a 4-round Feistel bijection with cycle walking,
 * applied to both endpoints.  Lists are sorted ascending by destination;
 * equal destinations keep generation order, so a payload drawn per
 * generated edge travels with it.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GEN_OK 0
#define GEN_EINVAL 1
#define GEN_ENOMEM 2

enum { TAG_SPLIT = 1, TAG_DST = 2, TAG_PAYLOAD = 3, TAG_PERM = 4, TAG_UNIF = 5, TAG_GEOM = 6 };

static inline uint64_t sm64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
/* one 64-bit draw for (seed, tag, entity, counter) */
static inline uint64_t draw(uint64_t seed, uint64_t tag, uint64_t ent, uint64_t ctr) {
  uint64_t k = sm64(seed ^ (tag * 0xd1b54a32d192ed03ULL));
  k = sm64(k ^ ent);
  return sm64(k ^ (ctr * 0x9e3779b97f4a7c15ULL));
}
/* uniform double in (0, 1] from the top 53 bits */
static inline double unif01c(uint64_t r) { return ((double)(r >> 11) + 1.0) * (1.0 / 9007199254740992.0); }

/* ---------------- Feistel permutation on [0, n) ---------------- */
typedef struct { uint64_t n; int half; uint64_t mask; uint64_t key[4]; } perm_t;

static void perm_init(perm_t *p, uint64_t n, uint64_t seed) {
  int bits = 1;
  while ((1ULL << bits) < n) bits++;
  p->half = (bits + 1) / 2;
  p->mask = (1ULL << p->half) - 1;
  p->n = n;
  for (int r = 0; r < 4; r++) p->key[r] = draw(seed, TAG_PERM, 0, (uint64_t)r);
}
static inline uint64_t feistel_fwd(const perm_t *p, uint64_t x) {
  uint64_t l = x >> p->half, r = x & p->mask;
  for (int i = 0; i < 4; i++) {
    uint64_t f = sm64(r ^ p->key[i]) & p->mask;
    uint64_t nl = r, nr = l ^ f;
    l = nl; r = nr;
  }
  return (l << p->half) | r;
}
static inline uint64_t feistel_inv(const perm_t *p, uint64_t x) {
  uint64_t l = x >> p->half, r = x & p->mask;
  for (int i = 3; i >= 0; i--) {
    uint64_t pl = r ^ (sm64(l ^ p->key[i]) & p->mask), pr = l;
    l = pl; r = pr;
  }
  return (l << p->half) | r;
}
/* cycle walking keeps the bijection inside [0, n) */
static inline uint64_t perm_fwd(const perm_t *p, uint64_t x) {
  do { x = feistel_fwd(p, x); } while (x >= p->n);
  return x;
}
static inline uint64_t perm_inv(const perm_t *p, uint64_t x) {
  do { x = feistel_inv(p, x); } while (x >= p->n);
  return x;
}

int gtgen_perm(uint64_t n, uint64_t seed, int inverse, const int32_t *in, int32_t *out, int64_t count) {
  if (n == 0 || n > (1ULL << 31)) return GEN_EINVAL;
  perm_t p; perm_init(&p, n, seed);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; i++)
    out[i] = (int32_t)(inverse ? perm_inv(&p, (uint64_t)in[i]) : perm_fwd(&p, (uint64_t)in[i]));
  return GEN_OK;
}

/* ---------------- binomial draw ---------------- */
static int64_t binom(int64_t trials, double p, uint64_t r1, uint64_t r2) {
  if (trials <= 0 || p <= 0.0) return 0;
  if (p >= 1.0) return trials;
  if (p > 0.5) return trials - binom(trials, 1.0 - p, r1, r2);
  if (trials <= 1000) {
    /* inversion: walk the CDF from k = 0 */
    double q = 1.0 - p, u = unif01c(r1), pmf = pow(q, (double)trials), cdf = pmf;
    int64_t k = 0;
    double ratio = p / q;
    while (cdf < u && k < trials) {
      pmf *= ratio * (double)(trials - k) / (double)(k + 1);
      k++;
      cdf += pmf;
    }
    return k;
  }
  double mu = (double)trials * p, sd = sqrt(mu * (1.0 - p));
  double u1 = unif01c(r1), u2 = unif01c(r2);
  double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  double k = floor(mu + sd * z + 0.5);
  if (k < 0) k = 0;
  if (k > (double)trials) k = (double)trials;
  return (int64_t)k;
}

/* admissible R-MAT source mass below `limit` inside a node with `j` free bits,
 * relative to the node's full mass (p1 = probability of a source one-bit) */
static double rmat_mass(int j, int64_t limit, double p1) {
  double w = 1.0, acc = 0.0;
  /* walk the path of `limit` from the top free bit down */
  for (int bit = j - 1; bit >= 0; bit--) {
    if (limit <= 0) return acc;
    int64_t halfsz = 1LL << bit;
    if (limit >= 2 * halfsz) return acc + w;
    if (limit > halfsz) {      /* lower half fully inside, continue in upper */
      acc += w * (1.0 - p1);
      w *= p1;
      limit -= halfsz;
    } else {                   /* only part of the lower half is inside */
      w *= (1.0 - p1);
    }
  }
  return acc + (limit > 0 ? w : 0.0);
}

/* probability that an edge of the node [lo, lo + 2^j) goes to its upper half */
static double split_prob(int64_t lo, int j, int64_t n, double p1) {
  int64_t half = 1LL << (j - 1);
  if (lo + 2 * half <= n) return p1;   /* node fully admissible */
  double ml = (1.0 - p1) * rmat_mass(j - 1, n - lo, p1);
  double mu = p1 * rmat_mass(j - 1, n - lo - half, p1);
  return (ml + mu) > 0 ? mu / (ml + mu) : 0.0;
}

/* Recursive split of `cnt` edges over the sources [lo, lo + 2^j) clipped at n. */
static void rmat_split(int64_t lo, int j, int64_t cnt, int64_t n, double p1, uint64_t seed,
                       int64_t *counts) {
  if (cnt == 0 || lo >= n) return;
  if (j == 0) { counts[lo] = cnt; return; }
  int64_t half = 1LL << (j - 1);
  double pu = split_prob(lo, j, n, p1);
  uint64_t node = ((uint64_t)j << 40) ^ (uint64_t)lo;
  int64_t up = binom(cnt, pu, draw(seed, TAG_SPLIT, node, 0), draw(seed, TAG_SPLIT, node, 1));
  rmat_split(lo, j - 1, cnt - up, n, p1, seed, counts);
  rmat_split(lo + half, j - 1, up, n, p1, seed, counts);
}

/* Top levels serially, then independent subtrees in parallel. */
static void rmat_counts(int64_t n, int scale, int64_t m, double p1, uint64_t seed, int64_t *counts) {
  memset(counts, 0, sizeof(int64_t) * (size_t)n);
  int top = scale < 12 ? scale : 12;
  int64_t nsub = 1LL << top;
  int64_t *sub = (int64_t *)calloc((size_t)nsub, sizeof(int64_t));
  /* breadth-first over the top `top` levels */
  sub[0] = m;
  for (int lvl = 0; lvl < top; lvl++) {
    int j = scale - lvl;                 /* free bits at this level's nodes */
    int64_t nodes = 1LL << lvl;
    for (int64_t i = nodes - 1; i >= 0; i--) {
      int64_t lo = i << j, cnt = sub[i];
      int64_t half = 1LL << (j - 1);
      int64_t up = 0;
      if (cnt > 0 && lo < n) {
        double pu = split_prob(lo, j, n, p1);
        (void)half;
        uint64_t node = ((uint64_t)j << 40) ^ (uint64_t)lo;
        up = binom(cnt, pu, draw(seed, TAG_SPLIT, node, 0), draw(seed, TAG_SPLIT, node, 1));
      }
      sub[2 * i] = cnt - up;
      sub[2 * i + 1] = up;
    }
  }
  int j = scale - top;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < nsub; i++) rmat_split(i << j, j, sub[i], n, p1, seed, counts);
  free(sub);
}

/* stable insertion/merge sort of (dst, payload) pairs by dst */
typedef struct { int32_t d; uint32_t p; } pair_t;
static void sort_pairs(pair_t *a, int64_t len, pair_t *tmp) {
  if (len <= 32) {
    for (int64_t i = 1; i < len; i++) {
      pair_t x = a[i];
      int64_t k = i - 1;
      while (k >= 0 && a[k].d > x.d) { a[k + 1] = a[k]; k--; }
      a[k + 1] = x;
    }
    return;
  }
  int64_t h = len / 2;
  sort_pairs(a, h, tmp);
  sort_pairs(a + h, len - h, tmp);
  int64_t i = 0, k = h, o = 0;
  while (i < h && k < len) tmp[o++] = (a[k].d < a[i].d) ? a[k++] : a[i++];
  while (i < h) tmp[o++] = a[i++];
  while (k < len) tmp[o++] = a[k++];
  memcpy(a, tmp, sizeof(pair_t) * (size_t)len);
}

static inline uint32_t payload_word(uint64_t r) {
  float f = (float)((double)(r >> 40) * (1.0 / 16777216.0)); /* exact: 24-bit fraction */
  uint32_t u; memcpy(&u, &f, 4); return u;
}

/* family codes */
#define FAM_RMAT 0
#define FAM_UNIFORM 1
#define FAM_GEOMETRIC 2

typedef struct {
  int family; int64_t n; int scale; int64_t ef;
  double a, b, c, d, p_geom; uint64_t seed; int permute;
} spec_t;

/* out-degree of ORIGINAL source u (before permutation) */
static int64_t *original_counts(const spec_t *s) {
  int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(s->n > 0 ? s->n : 1));
  if (!cnt) return NULL;
  if (s->family == FAM_RMAT) {
    rmat_counts(s->n, s->scale, s->ef * s->n, s->c + s->d, s->seed, cnt);
  } else {
    for (int64_t u = 0; u < s->n; u++) cnt[u] = s->ef;
  }
  return cnt;
}

/* Offsets of the generated CSR (after the optional permutation). */
int gtgen_offsets(int family, int64_t n, int scale, int64_t ef, double a, double b, double c, double d,
                  double p_geom, uint64_t seed, int permute, int64_t *O) {
  if (n < 0 || n > 2147483647LL || ef < 0) return GEN_EINVAL;
  if (family == FAM_RMAT && (scale < 0 || scale > 31 || (n > 0 && (1LL << scale) < n))) return GEN_EINVAL;
  O[0] = 0;
  if (n == 0) return GEN_OK;
  spec_t s = {family, n, scale, ef, a, b, c, d, p_geom, seed, permute};
  int64_t *cnt = original_counts(&s);
  if (!cnt) return GEN_ENOMEM;
  perm_t p; perm_init(&p, (uint64_t)n, seed);
  for (int64_t w = 0; w < n; w++) {
    int64_t u = permute ? (int64_t)perm_inv(&p, (uint64_t)w) : w;
    O[w + 1] = O[w] + cnt[u];
  }
  free(cnt);
  return GEN_OK;
}

/* Fill D (and P when non-NULL) for the offsets produced by gtgen_offsets. */
int gtgen_fill(int family, int64_t n, int scale, int64_t ef, double a, double b, double c, double d,
               double p_geom, uint64_t seed, int permute, const int64_t *O, int32_t *D, uint32_t *P) {
  (void)ef;
  if (n <= 0) return GEN_OK;
  perm_t p; perm_init(&p, (uint64_t)n, seed);
  double pd0 = b / (a + b), pd1 = d / (c + d); /* P(dst bit = 1 | src bit) */
  uint64_t thr0 = (uint64_t)(pd0 * 2097152.0), thr1 = (uint64_t)(pd1 * 2097152.0); /* 21-bit */
  double lq = (family == FAM_GEOMETRIC) ? log(1.0 - p_geom) : 1.0;
  int err = GEN_OK;
#pragma omp parallel
  {
    pair_t *buf = NULL, *tmp = NULL; int64_t cap = 0;
#pragma omp for schedule(dynamic, 256)
    for (int64_t w = 0; w < n; w++) {
      int64_t beg = O[w], len = O[w + 1] - O[w];
      if (len == 0) continue;
      if (len > cap) {
        free(buf); free(tmp);
        cap = len < 1024 ? 1024 : len;
        buf = (pair_t *)malloc(sizeof(pair_t) * (size_t)cap);
        tmp = (pair_t *)malloc(sizeof(pair_t) * (size_t)cap);
        if (!buf || !tmp) { err = GEN_ENOMEM; cap = 0; continue; }
      }
      uint64_t u = permute ? perm_inv(&p, (uint64_t)w) : (uint64_t)w;
      for (int64_t j = 0; j < len; j++) {
        uint64_t v = 0;
        if (family == FAM_RMAT) {
          for (uint64_t attempt = 0;; attempt++) {
            v = 0;
            uint64_t ctr = ((uint64_t)j << 12) | ((attempt & 0xFF) << 4);
            uint64_t r = 0; int avail = 0;
            for (int bit = scale - 1; bit >= 0; bit--) {
              if (avail == 0) { r = draw(seed, TAG_DST, u, ctr++); avail = 3; }
              uint64_t x = r & 0x1FFFFF; r >>= 21; avail--;
              uint64_t sb = (u >> bit) & 1;
              uint64_t one = x < (sb ? thr1 : thr0);
              v |= one << bit;
            }
            if ((int64_t)v < n) break;
          }
        } else if (family == FAM_UNIFORM) {
          uint64_t r = draw(seed, TAG_UNIF, u, (uint64_t)j);
          v = (uint64_t)(((unsigned __int128)r * (unsigned __int128)(uint64_t)n) >> 64);
        } else {
          double uu = unif01c(draw(seed, TAG_GEOM, u, (uint64_t)j));
          uint64_t o = 1 + (uint64_t)floor(log(uu) / lq);
          v = (u + (o % (uint64_t)n)) % (uint64_t)n;
        }
        if (permute) v = perm_fwd(&p, v);
        buf[j].d = (int32_t)v;
        buf[j].p = P ? payload_word(draw(seed, TAG_PAYLOAD, u, (uint64_t)j)) : 0u;
      }
      sort_pairs(buf, len, tmp);
      for (int64_t j = 0; j < len; j++) {
        D[beg + j] = buf[j].d;
        if (P) P[beg + j] = buf[j].p;
      }
    }
    free(buf); free(tmp);
  }
  return err;
}

/* splitmix64 stream value, exported for tests of the generator itself */
uint64_t gtgen_draw(uint64_t seed, uint64_t tag, uint64_t ent, uint64_t ctr) { return draw(seed, tag, ent, ctr); }
