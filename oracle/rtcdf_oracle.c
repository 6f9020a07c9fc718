/*
 * rtcdf_oracle.c -- CPU oracle for Range-Tiled CDF sort (RT-CDF).
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * benchmark's CPU baseline, never by the product library.  It shares no code
 * with the HIP path.  Plain sequential C; every function is the paper's
 * definition written out (see rtcdf_oracle.h for the citations).
 *
 * Parity pins (tests/test_oracle.py): exhaustive brute force against a
 * library sort for every array of length <= 6 over ranges <= 4, random small
 * arrays, the paper's worked example of Sec. 3.1 (Table "Example of local
 * CDFs and tile offsets"), the H-P example of Sec. 2.2, and the invariants of
 * Lemmas 1-3 and Theorem 1 of Sec. 3.2.
 */
#include "rtcdf_oracle.h"

#include <stdlib.h>

static int check_range_args(int64_t minVal, int64_t maxVal) {
  /* Sec. 2.1: a known integer range [minVal, maxVal); R = maxVal - minVal > 0.
   * Keys are int32, so the range must lie within [INT32_MIN, INT32_MAX + 1]. */
  if (maxVal <= minVal) return ORC_INVALID_ARGUMENT;
  if (minVal < (int64_t)INT32_MIN) return ORC_INVALID_ARGUMENT;
  if (maxVal > (int64_t)INT32_MAX + 1) return ORC_INVALID_ARGUMENT;
  return ORC_OK;
}

int oracle_counts(const int32_t* A, uint64_t n, int64_t minVal, int64_t maxVal,
                  uint64_t* cnt) {
  int rc = check_range_args(minVal, maxVal);
  if (rc) return rc;
  if (n > 0 && (A == NULL || cnt == NULL)) return ORC_INVALID_ARGUMENT;
  uint64_t R = (uint64_t)(maxVal - minVal);
  if (cnt)
    for (uint64_t v = 0; v < R; v++) cnt[v] = 0;
  for (uint64_t i = 0; i < n; i++) {
    int64_t key = (int64_t)A[i];
    if (key < minVal || key >= maxVal) return ORC_KEY_OUT_OF_RANGE;
    cnt[(uint64_t)(key - minVal)] += 1;   /* c_v, v = A[i] - minVal */
  }
  return ORC_OK;
}

int oracle_sort(const int32_t* A, uint64_t n, int64_t minVal, int64_t maxVal,
                int32_t* B) {
  int rc = check_range_args(minVal, maxVal);
  if (rc) return rc;
  if (n == 0) return ORC_OK;
  if (A == NULL || B == NULL) return ORC_INVALID_ARGUMENT;
  uint64_t R = (uint64_t)(maxVal - minVal);
  uint64_t* cnt = (uint64_t*)malloc(R * sizeof(uint64_t));
  if (!cnt) return ORC_INVALID_ARGUMENT;
  rc = oracle_counts(A, n, minVal, maxVal, cnt);
  if (rc) { free(cnt); return rc; }
  /* Value v occupies [sum_{u<v} c_u, sum_{u<=v} c_u) (Sec. 2.1). */
  uint64_t start = 0;                    /* sum_{u<v} c_u */
  for (uint64_t v = 0; v < R; v++) {
    uint64_t end = start + cnt[v];       /* sum_{u<=v} c_u */
    for (uint64_t p = start; p < end; p++) B[p] = (int32_t)(minVal + (int64_t)v);
    start = end;
  }
  free(cnt);
  return start == n ? ORC_OK : ORC_INVALID_ARGUMENT;
}

int oracle_tile_intermediates(const int32_t* A, uint64_t n, int64_t minVal,
                              int64_t maxVal, uint64_t T, uint64_t* hist,
                              uint64_t* cdf, uint64_t* O) {
  int rc = check_range_args(minVal, maxVal);
  if (rc) return rc;
  if (T == 0) return ORC_INVALID_ARGUMENT;
  if (n > 0 && A == NULL) return ORC_INVALID_ARGUMENT;
  uint64_t R = (uint64_t)(maxVal - minVal);
  uint64_t m = (R + T - 1) / T;          /* m = ceil(R/T) */
  uint64_t* H = (uint64_t*)calloc(R, sizeof(uint64_t));
  if (!H) return ORC_INVALID_ARGUMENT;
  for (uint64_t i = 0; i < n; i++) {
    int64_t key = (int64_t)A[i];
    if (key < minVal || key >= maxVal) { free(H); return ORC_KEY_OUT_OF_RANGE; }
  }
  /* Alg. 5 for every tile: tile t counts only the keys whose normalised value
   * x = A[i] - minVal - b_t lies in [0, w_t). */
  for (uint64_t t = 0; t < m; t++) {
    uint64_t b = t * T;
    uint64_t w = (R - b < T) ? (R - b) : T;   /* w_t = min(T, R - b_t) */
    for (uint64_t i = 0; i < n; i++) {
      int64_t x = (int64_t)A[i] - minVal - (int64_t)b;
      if (x >= 0 && (uint64_t)x < w) H[b + (uint64_t)x] += 1;
    }
  }
  if (hist)
    for (uint64_t v = 0; v < R; v++) hist[v] = H[v];
  /* Alg. 4: in-place inclusive scan of each tile's slice -> local CDF. */
  for (uint64_t t = 0; t < m; t++) {
    uint64_t b = t * T;
    uint64_t w = (R - b < T) ? (R - b) : T;
    for (uint64_t x = 1; x < w; x++) H[b + x] += H[b + x - 1];
  }
  if (cdf)
    for (uint64_t v = 0; v < R; v++) cdf[v] = H[v];
  /* Alg. 6: O[t] = running total of the last local-CDF entries of the
   * preceding tiles. */
  if (O) {
    uint64_t offset = 0;
    for (uint64_t t = 0; t < m; t++) {
      uint64_t b = t * T;
      uint64_t w = (R - b < T) ? (R - b) : T;
      O[t] = offset;
      offset += H[b + w - 1];
    }
  }
  free(H);
  return ORC_OK;
}

int oracle_output_from_local_cdfs(const uint64_t* cdf, const uint64_t* O,
                                  int64_t minVal, int64_t maxVal, uint64_t T,
                                  uint64_t n, int32_t* B) {
  int rc = check_range_args(minVal, maxVal);
  if (rc) return rc;
  if (T == 0 || cdf == NULL || O == NULL) return ORC_INVALID_ARGUMENT;
  if (n > 0 && B == NULL) return ORC_INVALID_ARGUMENT;
  uint64_t R = (uint64_t)(maxVal - minVal);
  uint64_t m = (R + T - 1) / T;
  uint64_t written = 0;
  for (uint64_t t = 0; t < m; t++) {
    uint64_t b = t * T;
    uint64_t w = (R - b < T) ? (R - b) : T;
    const uint64_t* C = cdf + b;
    uint64_t tileStart = O[t];
    uint64_t tileCount = C[w - 1];
    if (tileStart + tileCount > n) return ORC_INVALID_ARGUMENT;
    for (uint64_t p = 0; p < tileCount; p++) {
      /* x = min{ j : C[j] >= p + 1 }, by bisection on the nondecreasing C. */
      uint64_t lo = 0, hi = w - 1;        /* C[w-1] = tileCount >= p + 1 */
      while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (C[mid] >= p + 1) hi = mid; else lo = mid + 1;
      }
      B[tileStart + p] = (int32_t)(minVal + (int64_t)(b + lo));
    }
    written += tileCount;
  }
  return written == n ? ORC_OK : ORC_INVALID_ARGUMENT;
}

int oracle_prefix_max_output(const uint64_t* P1, int64_t minVal, int64_t maxVal,
                             uint64_t n, int32_t* B) {
  int rc = check_range_args(minVal, maxVal);
  if (rc) return rc;
  if (P1 == NULL || (n > 0 && B == NULL)) return ORC_INVALID_ARGUMENT;
  uint64_t R = (uint64_t)(maxVal - minVal);
  if (P1[R - 1] != n) return ORC_INVALID_ARGUMENT;
  /* Work on normalised values, then re-offset by minVal. */
  uint64_t* Bn = (uint64_t*)calloc(n ? n : 1, sizeof(uint64_t));   /* B <- 0 */
  if (!Bn) return ORC_INVALID_ARGUMENT;
  for (uint64_t d = 1; d < R; d++)        /* a step of the CDF at d */
    if (P1[d] > P1[d - 1]) Bn[P1[d - 1]] = d;
  for (uint64_t i = 1; i < n; i++)        /* inclusive prefix maximum */
    if (Bn[i - 1] > Bn[i]) Bn[i] = Bn[i - 1];
  for (uint64_t i = 0; i < n; i++) B[i] = (int32_t)(minVal + (int64_t)Bn[i]);
  free(Bn);
  return ORC_OK;
}

void oracle_verify_begin(oracle_cursor_t* c, const uint64_t* cnt, uint64_t R,
                         int64_t minVal) {
  c->cnt = cnt;
  c->R = R;
  c->minVal = minVal;
  c->v = 0;
  c->left = R ? cnt[0] : 0;
  c->pos = 0;
}

int oracle_verify_chunk(oracle_cursor_t* c, const int32_t* Bchunk, uint64_t len,
                        uint64_t* bad_pos) {
  for (uint64_t i = 0; i < len; i++) {
    /* advance to the value that owns position c->pos (skips empty values) */
    while (c->left == 0 && c->v + 1 < c->R) {
      c->v += 1;
      c->left = c->cnt[c->v];
    }
    if (c->left == 0 ||
        (int64_t)Bchunk[i] != c->minVal + (int64_t)c->v) {
      if (bad_pos) *bad_pos = c->pos;
      return ORC_MISMATCH;
    }
    c->left -= 1;
    c->pos += 1;
  }
  return ORC_OK;
}

int oracle_verify_end(const oracle_cursor_t* c, uint64_t n) {
  return c->pos == n ? ORC_OK : ORC_MISMATCH;
}
