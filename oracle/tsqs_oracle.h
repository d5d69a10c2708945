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

/* Indices into oracle_counters_t.events: coverage of the states of SIII.B-F
 * and of the outcomes of the handlers of SIII.I. */
enum {
  OE_STATE1 = 0,        /* State 1 entered (SIII.B) */
  OE_CLOSE_BY_SIDE,     /* l or r met the zone (State 1's empty zone slot moved there) */
  OE_CLOSE_BY_ZONE,     /* the zone met l or r */
  OE_STATE2L, OE_STATE2R, OE_STATE3L, OE_STATE3R,   /* SIII.C choices */
  OE_ROLL,              /* State 2: the zone rolled by one slot (SIII.D) */
  OE_RUN_FITS,          /* State 3: a run of keys copied whole into the gap (SIII.E) */
  OE_RUN_FILLS,         /* State 3: the gap closed before the run ended */
  OE_COPY_BACK,         /* tar[] copied back (SIII.F) */
  OE_EXIT2,             /* temp and p put back (SIII.F) */
  OE_BYPASS,            /* stage ended with temp unused */
  OE_R_AT_MID,          /* initialization: every key right of mid above p (R7) */
  OE_SORTED, OE_SORTED_CONFIRMED, OE_SORTED_FALLBACK,             /* SIII.I */
  OE_REVERSED, OE_REV_SWAP, OE_REV_CONFIRMED, OE_REV_FALLBACK,    /* SIII.I */
  OE_COUNT
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
  uint64_t internal_errors; /* watchdog: a slot outside the stage, too many comparisons, tar[] overflow */
  uint64_t post_errors;     /* debug: a stage whose result is not a three-way partition
                               around its pivot of the multiset it was given */
  uint64_t events[32];      /* OE_* */
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

/* Median of five (SIII.H; reading R4) on ar5[0..4]: sorts them in place,
 * stores the median (ar5[2]) in *piv; returns 1 / -1 / 0 as MedianOf3S. */
int oracle_median5_i32(int32_t *ar5, int32_t *piv, oracle_counters_t *cnt);
/* The size-tiered pivot choice of SIII.H / SV.C on ar[0..n-1] (n >= 3) with
 * the tiers and jitter of prm (one generator step from prm->seed, as at the
 * start of a sort call): permutes the samples in place, stores the pivot in
 * *piv and returns the sorted / reversed flag. */
int oracle_choose_pivot_i32(int32_t *ar, size_t n, const oracle_params_t *prm, int32_t *piv,
                            oracle_counters_t *cnt);

/* Entry into the middle of a stage, for hand-traced checks of States 2L/2R,
 * 3L/3R and exit2 (SIII.D-F).  The caller gives the array, the pointers, the
 * pivot p, temp, the two empty slots, and for States 2 / 3 the comparison lc
 * of the key m stands on (m_scan..._2 of the paper: the entry after SIII.C).
 * The state runs to its end, then exit2; l and r come back as the bounds of
 * the children [a..l] and [r..b].  Empty slots are checked (hole_errors). */
enum { OR_STATE2 = 0, OR_STATE3 = 1, OR_EXIT2 = 2 };
typedef struct {
  int64_t a, b, l, r, m, ml, mr;
  int64_t hole0, hole1;     /* the two empty slots at entry */
  int32_t entry;            /* OR_* */
  int32_t open_side;        /* 0: m moves toward l (2L, 3L); 1: toward r (2R, 3R) */
  int32_t lc;               /* cmp(ar[m], p) at entry (States 2 and 3) */
  int32_t p, temp;
  int32_t reserved;
} oracle_entry_t;
int oracle_run_entry_i32(int32_t *ar, size_t n, oracle_entry_t *e, oracle_counters_t *cnt);

#ifdef __cplusplus
}
#endif
#endif
