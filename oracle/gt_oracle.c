/*
 * ORACLE — test infrastructure only.  Nothing on the product path may link,
 * load or call this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.
 *
 * Plain sequential CSR -> CSC graph transposition: Algorithm 1 (Atomic GT,
 * Section II-B) executed by a single thread, so every fetch-and-add returns
 * in edge order and each transposed neighbour list comes out in increasing
 * CSR edge position, i.e. ascending source with multi-edges in CSR order.
 * CSR/CSC follow the definitions of Section II-A: offsets has |V|+1 entries;
 * CSR edges hold destinations, CSC edges hold sources; an edge weight (here a
 * 32-bit payload word) travels with its edge unchanged.
 *
 * Counters are 64-bit, so no narrow-counter carry is needed here.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_EGRAPH 2
#define ORC_ENOMEM 3
#define ORC_EINTERNAL 4

/* A CSR is valid when offsets[0] = 0, offsets is nondecreasing,
 * offsets[n] = m and every destination lies in [0, n). */
int gt_oracle_validate(int64_t n, int64_t m, const int64_t *O, const int32_t *D) {
  if (n < 0 || m < 0) return ORC_EINVAL;
  if (O[0] != 0 || O[n] != m) return ORC_EGRAPH;
  for (int64_t u = 0; u < n; u++)
    if (O[u + 1] < O[u]) return ORC_EGRAPH;
  for (int64_t e = 0; e < m; e++)
    if (D[e] < 0 || (int64_t)D[e] >= n) return ORC_EGRAPH;
  return ORC_OK;
}

/* Full transposition.  T: int64[n+1], S: int32[m], Q: uint32[m] (ignored when
 * P is NULL). */
int gt_oracle_transpose(int64_t n, int64_t m, const int64_t *O, const int32_t *D, const uint32_t *P,
                        int64_t *T, int32_t *S, uint32_t *Q) {
  int rc = gt_oracle_validate(n, m, O, D);
  if (rc != ORC_OK) return rc;
  /* Step 1: in-degree of every vertex (Alg. 1, counters). */
  uint64_t *cnt = (uint64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
  if (!cnt) return ORC_ENOMEM;
  for (int64_t e = 0; e < m; e++) cnt[D[e]]++;
  /* Step 2: t_offsets = exclusive prefix sum; IP starts as a copy. */
  T[0] = 0;
  for (int64_t v = 0; v < n; v++) T[v + 1] = T[v] + (int64_t)cnt[v];
  for (int64_t v = 0; v < n; v++) cnt[v] = (uint64_t)T[v];
  /* Step 3: walk the sources in order; each edge takes the next slot of its
   * destination's list. */
  for (int64_t u = 0; u < n; u++) {
    for (int64_t e = O[u]; e < O[u + 1]; e++) {
      uint64_t p = cnt[D[e]]++;
      S[p] = (int32_t)u;
      if (P) Q[p] = P[e];
    }
  }
  /* Footnote 1: after Step 3 every insertion point equals the next offset. */
  for (int64_t v = 0; v < n; v++)
    if ((int64_t)cnt[v] != T[v + 1]) { free(cnt); return ORC_EINTERNAL; }
  free(cnt);
  return ORC_OK;
}

/* The same computation restricted to the destinations [lo, hi): fills
 * T[lo..hi] (written to Tslice[0..hi-lo]) and the lists of those vertices
 * (written from Sslice[0], Qslice[0]; their length is T[hi]-T[lo]).  Needs
 * O(hi-lo) memory besides the slices, so full-size inputs can be checked on
 * chosen vertex ranges. */
int gt_oracle_transpose_slice(int64_t n, int64_t m, const int64_t *O, const int32_t *D, const uint32_t *P,
                              int64_t lo, int64_t hi, int64_t *Tslice, int32_t *Sslice, uint32_t *Qslice) {
  if (n < 0 || m < 0 || lo < 0 || hi > n || lo > hi) return ORC_EINVAL;
  int64_t w = hi - lo;
  uint64_t *cnt = (uint64_t *)calloc((size_t)(w > 0 ? w : 1), sizeof(uint64_t));
  if (!cnt) return ORC_ENOMEM;
  int64_t below = 0;
  for (int64_t e = 0; e < m; e++) {
    int64_t v = D[e];
    if (v < 0 || v >= n) { free(cnt); return ORC_EGRAPH; }
    if (v < lo) below++;
    else if (v < hi) cnt[v - lo]++;
  }
  Tslice[0] = below;
  for (int64_t i = 0; i < w; i++) Tslice[i + 1] = Tslice[i] + (int64_t)cnt[i];
  for (int64_t i = 0; i < w; i++) cnt[i] = (uint64_t)(Tslice[i] - below);
  for (int64_t u = 0; u < n; u++) {
    for (int64_t e = O[u]; e < O[u + 1]; e++) {
      int64_t v = D[e];
      if (v < lo || v >= hi) continue;
      uint64_t p = cnt[v - lo]++;
      Sslice[p] = (int32_t)u;
      if (P) Qslice[p] = P[e];
    }
  }
  free(cnt);
  return ORC_OK;
}
