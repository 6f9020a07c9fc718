/*
 * rtcdf_oracle.h -- CPU oracle for Range-Tiled CDF sort (RT-CDF).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no header, type, helper or constant with the HIP
 * path.
 *
 * Everything here is plain, sequential and slow on purpose: each function is
 * the definition the paper gives, written out, so that a reader can check it
 * against the paper by eye.  Sections cited are those of the paper
 * "Shared-Memory Range-Tiled CDF Sort for Small-Range Integer Keys on GPUs".
 *
 * Conventions (readings of the paper where it leaves a choice open):
 *   - keys are int32, the range is the half-open [minVal, maxVal) (Sec. 2.1);
 *     minVal/maxVal are int64 so that maxVal = 2^31 is expressible;
 *   - R = maxVal - minVal; the paper subtracts minVal "for notation" only
 *     (Sec. 2.1), so outputs carry the original key values;
 *   - counts are uint64 (no overflow is possible for any n that fits memory).
 *
 * Return codes: 0 on success, otherwise one of the ORC_ codes below.
 */
#ifndef RTCDF_ORACLE_H
#define RTCDF_ORACLE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_INVALID_ARGUMENT 1   /* NULL pointer with n > 0, maxVal <= minVal, bad T */
#define ORC_KEY_OUT_OF_RANGE 2   /* a key outside [minVal, maxVal) */
#define ORC_MISMATCH 3           /* verifier found a difference */

/* Sec. 2.1: c_v = number of occurrences of value v, for v = key - minVal in
 * [0, R).  cnt must hold R entries and is overwritten. */
int oracle_counts(const int32_t* A, uint64_t n, int64_t minVal, int64_t maxVal,
                  uint64_t* cnt);

/* Sec. 2.1: the sorted output.  Value v occupies the output interval
 * [sum_{u<v} c_u, sum_{u<=v} c_u); B receives minVal + v there.  B must hold n
 * entries and must not alias A.  This is the plain definition of the result
 * RT-CDF computes (Theorem 1), not the tiled method. */
int oracle_sort(const int32_t* A, uint64_t n, int64_t minVal, int64_t maxVal,
                int32_t* B);

/* Sec. 3 (tile geometry) and Alg. 4-6: the intermediates of RT-CDF for tile
 * width T.  m = ceil(R/T); tile t covers [b_t, b_t + w_t) with b_t = t*T and
 * w_t = min(T, R - b_t).
 *   hist[R]: hist[b_t + x] = number of keys equal to minVal + b_t + x
 *            (Alg. 5, the per-tile histogram);
 *   cdf[R] : per-tile inclusive prefix sum of hist (Alg. 4, local CDF);
 *   O[m]   : O[t] = sum of the totals of tiles 0..t-1, accumulated tile by
 *            tile as in Alg. 6.
 * Any of the three output pointers may be NULL. */
int oracle_tile_intermediates(const int32_t* A, uint64_t n, int64_t minVal,
                              int64_t maxVal, uint64_t T, uint64_t* hist,
                              uint64_t* cdf, uint64_t* O);

/* Alg. 7, applied to every tile: given the local CDFs and tile offsets, for
 * each within-tile position p the value is b_t + min{ j : C_t[j] >= p + 1 },
 * written at B[O[t] + p].  n is the total number of keys.  Used to check that
 * the tiled method reaches the plain definition. */
int oracle_output_from_local_cdfs(const uint64_t* cdf, const uint64_t* O,
                                  int64_t minVal, int64_t maxVal, uint64_t T,
                                  uint64_t n, int32_t* B);

/* Alg. 3 (RefHP output generation): B <- 0; for d in [1,R) with
 * P1[d] > P1[d-1]: B[P1[d-1]] <- d; then the inclusive prefix maximum of B.
 * P1 is the full-range CDF (inclusive prefix sum of the counts).  Output
 * values are re-offset by minVal.  B must hold n entries. */
int oracle_prefix_max_output(const uint64_t* P1, int64_t minVal, int64_t maxVal,
                             uint64_t n, int32_t* B);

/* Streaming check of a sorted output against counts, for arrays too large to
 * hold a second copy.  The cursor walks the expansion of cnt in value order:
 * call oracle_verify_begin once, then oracle_verify_chunk on consecutive
 * chunks of the candidate output, then oracle_verify_end.  Returns ORC_OK if
 * every element seen so far equals the plain definition's element at the same
 * position; on the first difference it returns ORC_MISMATCH and stores the
 * global position in *bad_pos. */
typedef struct {
  const uint64_t* cnt;
  uint64_t R;
  int64_t minVal;
  uint64_t v;          /* current value (offset from minVal) */
  uint64_t left;       /* copies of v still expected */
  uint64_t pos;        /* global position of the next element */
} oracle_cursor_t;

void oracle_verify_begin(oracle_cursor_t* c, const uint64_t* cnt, uint64_t R,
                         int64_t minVal);
int oracle_verify_chunk(oracle_cursor_t* c, const int32_t* Bchunk, uint64_t len,
                        uint64_t* bad_pos);
int oracle_verify_end(const oracle_cursor_t* c, uint64_t n);

#ifdef __cplusplus
}
#endif
#endif
