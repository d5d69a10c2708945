/*
 * exhaustive.c -- brute-force pin of the Triple State QuickSort oracle.
 *
 * For every sequence of length n (1 <= n <= nmax) over the alphabet {0..n-1}
 * (sum of n^n sequences: 17,650,828 for nmax = 8, which contains every weak
 * ordering of up to 8 keys), sorts (key, id) pairs with the oracle and checks:
 *   - the keys equal the counting sort of the input (the plain definition of
 *     the result: the unique non-decreasing arrangement of the multiset);
 *   - the ids form a permutation and key_in[id_out[i]] == key_out[i];
 *   - no empty-slot misuse (hole_errors == 0), no comparison touching an
 *     element of a finished equal band (revisit_errors == 0, the paper's
 *     "never compared again", SIII), tar[] never above n/2 (SIII.G), every
 *     stage's result a three-way partition of its own keys (post_errors ==
 *     0), and no internal error.
 * Prints one JSON line with totals and per-event counts (coverage of the
 * states and handler outcomes).
 *
 * Usage: exhaustive NMAX INS_MAX MED3_BELOW MEDOF3_SMALL HANDLERS TOL SEED [KEYS_ONLY]
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "tsqs_oracle.h"

int main(int argc, char **argv) {
  int nmax, n, i;
  oracle_params_t q;
  oracle_counters_t c;
  uint64_t arrays = 0, bad_keys = 0, bad_ids = 0, hole = 0, revisit = 0, internal = 0,
           tar_over = 0, rc_bad = 0, comps = 0, copies = 0, post = 0;
  uint64_t hits[64];
  int keys_only = 0;
  if (argc < 8) {
    fprintf(stderr, "usage: %s NMAX INS_MAX MED3_BELOW MEDOF3_SMALL HANDLERS TOL SEED [KEYS_ONLY]\n", argv[0]);
    return 2;
  }
  nmax = atoi(argv[1]);
  oracle_default_params(&q);
  q.ins_max = atoi(argv[2]);
  q.med3_below = atoi(argv[3]);
  q.medof3_small = atoi(argv[4]);
  q.handlers = atoi(argv[5]);
  q.reverse_tolerance = atoi(argv[6]);
  q.seed = (uint32_t)strtoul(argv[7], NULL, 10);
  if (argc > 8) keys_only = atoi(argv[8]);
  /* keep every part of <= 8 keys in the median-of-3 / median-of-5 tiers */
  q.med5_below = 1000;
  q.ninther_below = 2000;
  q.debug_checks = keys_only ? 0 : 1;
  memset(hits, 0, sizeof hits);

  for (n = 1; n <= nmax; n++) {
    int digits[16];
    int32_t kin[16], kout[16], kref[16];
    uint32_t ids[16];
    memset(digits, 0, sizeof digits);
    for (;;) {
      int hist[16], seen[16], j, pos, ok = 1;
      int rc;
      for (i = 0; i < n; i++) { kin[i] = digits[i]; kout[i] = digits[i]; ids[i] = (uint32_t)i; }
      if (keys_only) rc = oracle_tsqs_sort_i32(kout, (size_t)n, &q, &c);
      else rc = oracle_tsqs_sort_pairs_i32(kout, ids, (size_t)n, &q, &c);
      arrays++;
      if (rc != 0) rc_bad++;
      /* counting sort = the plain definition */
      memset(hist, 0, sizeof hist);
      for (i = 0; i < n; i++) hist[kin[i]]++;
      for (j = 0, pos = 0; j < n; j++) while (hist[j]-- > 0) kref[pos++] = j;
      for (i = 0; i < n; i++) if (kout[i] != kref[i]) ok = 0;
      if (!ok) {
        if (bad_keys < 5) {
          fprintf(stderr, "BAD KEYS n=%d in:", n);
          for (i = 0; i < n; i++) fprintf(stderr, " %d", kin[i]);
          fprintf(stderr, " out:");
          for (i = 0; i < n; i++) fprintf(stderr, " %d", kout[i]);
          fprintf(stderr, "\n");
        }
        bad_keys++;
      }
      if (!keys_only) {
        memset(seen, 0, sizeof seen);
        ok = 1;
        for (i = 0; i < n; i++) {
          if (ids[i] >= (uint32_t)n || seen[ids[i]]) { ok = 0; break; }
          seen[ids[i]] = 1;
          if (kin[ids[i]] != kout[i]) { ok = 0; break; }
        }
        if (!ok) bad_ids++;
      }
      hole += c.hole_errors;
      revisit += c.revisit_errors;
      internal += c.internal_errors;
      if (c.tar_peak > (uint64_t)(n / 2)) tar_over++;
      comps += c.comparisons;
      copies += c.copies;
      post += c.post_errors;
      for (i = 0; i < OE_COUNT; i++) hits[i] += c.events[i];
      if ((hole || revisit || internal) && (hole + revisit + internal) < 4 && c.hole_errors + c.revisit_errors + c.internal_errors) {
        fprintf(stderr, "CHECK FAIL n=%d hole=%llu rev=%llu int=%llu in:", n,
                (unsigned long long)c.hole_errors, (unsigned long long)c.revisit_errors,
                (unsigned long long)c.internal_errors);
        for (i = 0; i < n; i++) fprintf(stderr, " %d", kin[i]);
        fprintf(stderr, "\n");
      }
      /* next sequence (odometer in base n) */
      for (pos = 0; pos < n; pos++) {
        if (++digits[pos] < n) break;
        digits[pos] = 0;
      }
      if (pos == n) break;
    }
  }
  printf("{\"arrays\": %llu, \"bad_keys\": %llu, \"bad_ids\": %llu, \"hole_errors\": %llu, "
         "\"revisit_errors\": %llu, \"internal_errors\": %llu, \"tar_over\": %llu, "
         "\"rc_bad\": %llu, \"post_errors\": %llu, \"comparisons\": %llu, \"copies\": %llu, "
         "\"hits\": [",
         (unsigned long long)arrays, (unsigned long long)bad_keys, (unsigned long long)bad_ids,
         (unsigned long long)hole, (unsigned long long)revisit, (unsigned long long)internal,
         (unsigned long long)tar_over, (unsigned long long)rc_bad, (unsigned long long)post,
         (unsigned long long)comps,
         (unsigned long long)copies);
  for (i = 0; i < OE_COUNT; i++) printf("%s%llu", i ? ", " : "", (unsigned long long)hits[i]);
  printf("]}\n");
  oracle_free_storage();
  return 0;
}
