/*
 * tsqs_oracle.h -- CPU oracle for Triple State QuickSort (Muqaddas, "Triple State
 * QuickSort, A replacement for the C/C++ library qsort", arXiv 1505.00558).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, single-threaded
 * reference that the GPU library is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or helper with the GPU path and must never be used to
 * produce a product result.
 *
 * What it computes: the unique non-decreasing arrangement of the input keys
 * under a total order (integers: the usual order; float32: IEEE 754-2008
 * totalOrder on the bit patterns), reached by the array-based form of the
 * paper's algorithm: size-tiered pivot selection (paper SIII.H, SIII.I, SV.C),
 * the possibly-sorted / possibly-reversed handlers (SIII.I), the State 1 /
 * 2L / 2R / 3L / 3R partition state machine with copy-back (SIII.A-F),
 * insertion sort for tiny parts (SIV) and the n/2 temporary buffer (SIII.G).
 * Every comparison and element copy is counted (SV.A: virtual swaps =
 * copies / 3).
 *
 * Readings of passages the paper leaves out (its "complete code" is not part of
 * the paper) are listed in the design doc; each is also named at the point of use in
 * tsqs_stage.inc.
 *
 * Parity status of each function is stated in tsqs_oracle.c.
 */
#ifndef TSQS_ORACLE_H
#define TSQS_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Tunables.  Integer fields so that ctypes can mirror the struct exactly. */
typedef struct {
  int32_t ins_max;           /* insertion sort when the part has <= ins_max elements (>= 2) */
  int32_t med3_below;        /* median of 3 when n' < med3_below (only if medof3_small) */
  int32_t med5_below;        /* median of 5 when n' < med5_below */
  int32_t ninther_below;     /* ninther when n' < ninther_below, fifteenther otherwise */
  int32_t medof3_small;      /* the paper's MEDOF3_SMALL directive (SV.C) */
  int32_t random_samples;    /* the paper's RANDOM_SAMPLES directive (SV.C) */
  int32_t handlers;          /* possibly-sorted / possibly-reversed handlers (SIII.I) */
  int32_t reverse_tolerance; /* REVERSE_TOLERANCE of the reversed handler (SIII.I) */
  int32_t analysis_random_pivot; /* analysis mode of SV.A: one random pivot, no handlers */
  int32_t debug_checks;      /* hole shadow + never-revisited tags (pairs only) */
  uint32_t seed;             /* seed of the internal Park-Miller generator (SV.C) */
  int32_t reserved;
} oracle_params_t;

/* Indices into oracle_counters_t.label_hits (one per state / handler branch). */
enum {
  OL_MAIN_INIT = 0, OL_MAIN_R_AT_MID, OL_L_SCAN1, OL_L_EQ1, OL_L_GT1, OL_R_SCAN1,
  OL_R_EQ1, OL_R_LT1, OL_MR_SCAN1, OL_MR_FOUND1, OL_ML_SCAN1, OL_ML_FOUND1,
  OL_CLOSE_LEFT_CHECKM, OL_CLOSE_LEFT, OL_CLOSE_LEFT_NOSCAN, OL_CLOSE_RIGHT_CHECKM,
  OL_CLOSE_RIGHT, OL_CLOSE_RIGHT_NOSCAN, OL_M_SCAN2L, OL_M_FOUND2L, OL_L_SCAN2L,
  OL_M_SCAN2R, OL_M_FOUND2R, OL_R_SCAN2R, OL_M_SCAN3L, OL_M_EQ3L, OL_M_FOUND3L,
  OL_M_LT3L, OL_L_SCAN3L, OL_M_SCAN3R, OL_M_EQ3R, OL_M_FOUND3R, OL_M_GT3R,
  OL_R_SCAN3R, OL_EXIT3L, OL_EXIT3R, OL_EXIT2, OL_BYPASS, OL_SORTED, OL_SORTED_EQ,
  OL_SORTED_GT, OL_REVERSED, OL_REV_SWAP, OL_REV_GT_GT, OL_REV_GT_EQ, OL_REV_LT,
  OL_REV_EQ, OL_REV_LEFT_DONE, OL_RUN3L_LONG, OL_RUN3R_LONG, OL_REV_FALLBACK,
  OL_COUNT
};

typedef struct {
  uint64_t comparisons;     /* calls of the three-valued compare */
  uint64_t copies;          /* element copies into/out of ar, tar, p, temp (SV.A) */
  uint64_t pivot_copies;    /* the subset of copies that load the pivot p */
  uint64_t literal_swaps;   /* swaps done by the reversed handler (3 copies each) */
  uint64_t stages;          /* partitioning stages */
  uint64_t insertion_stages;
  uint64_t max_depth;
  uint64_t tar_peak;        /* largest fill of tar[] in one stage */
  uint64_t hole_errors;     /* debug: read of an empty slot / overwrite of a live slot */
  uint64_t revisit_errors;  /* debug: comparison touching a finalized element */
  uint64_t internal_errors; /* watchdog or invariant failure */
  uint64_t label_hits[64];
} oracle_counters_t;

void oracle_default_params(oracle_params_t *prm);
/* Releases the persistent temporary buffers (the paper's
 * FreeTripleStateQuickSortStorage(), SIII.G). */
void oracle_free_storage(void);

/* Sort n keys in place.  prm may be NULL (defaults), cnt may be NULL.
 * Returns 0, -1 on invalid parameters, -2 on an internal error (counted). */
int oracle_tsqs_sort_i32(int32_t *keys, size_t n, const oracle_params_t *prm, oracle_counters_t *cnt);
int oracle_tsqs_sort_u32(uint32_t *keys, size_t n, const oracle_params_t *prm, oracle_counters_t *cnt);
int oracle_tsqs_sort_i64(int64_t *keys, size_t n, const oracle_params_t *prm, oracle_counters_t *cnt);
int oracle_tsqs_sort_u64(uint64_t *keys, size_t n, const oracle_params_t *prm, oracle_counters_t *cnt);
/* float32 keys passed as their bit patterns, ordered by IEEE 754-2008 totalOrder */
int oracle_tsqs_sort_f32(uint32_t *keys, size_t n, const oracle_params_t *prm, oracle_counters_t *cnt);

/* Sort (key, payload) elements by key; payloads travel with their keys. */
int oracle_tsqs_sort_pairs_i32(int32_t *keys, uint32_t *vals, size_t n, const oracle_params_t *prm, oracle_counters_t *cnt);
int oracle_tsqs_sort_pairs_u32(uint32_t *keys, uint32_t *vals, size_t n, const oracle_params_t *prm, oracle_counters_t *cnt);
int oracle_tsqs_sort_pairs_i64(int64_t *keys, uint32_t *vals, size_t n, const oracle_params_t *prm, oracle_counters_t *cnt);
int oracle_tsqs_sort_pairs_u64(uint64_t *keys, uint32_t *vals, size_t n, const oracle_params_t *prm, oracle_counters_t *cnt);
int oracle_tsqs_sort_pairs_f32(uint32_t *keys, uint32_t *vals, size_t n, const oracle_params_t *prm, oracle_counters_t *cnt);

/* Test hooks for the two complete listings of the paper. */
/* MedianOf3S (SIII.I) on ar3[0..2]: sorts them in place, stores the median in
 * *piv and returns 1 (were non-decreasing), -1 (strictly decreasing) or 0. */
int oracle_median3_i32(int32_t *ar3, int32_t *piv, oracle_counters_t *cnt);
/* Insertion sort with direct copies (SIV) on ar[0..n-1]. */
int oracle_insertion_i32(int32_t *ar, size_t n, oracle_counters_t *cnt);

#ifdef __cplusplus
}
#endif
#endif
