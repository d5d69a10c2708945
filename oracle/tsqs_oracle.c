/*
 * tsqs_oracle.c -- CPU oracle for Triple State QuickSort (arXiv 1505.00558).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark.  Shares nothing with the GPU library.
 *
 * Parity status of the functions exported here:
 *   oracle_tsqs_sort_* / _pairs_*  output keys pinned by brute force over every
 *        sequence of length <= 8 (tests/native/exhaustive.c), by library sorts
 *        on large inputs, by the totalOrder fixture for float32, and by the
 *        stage postcondition / never-revisited / hole / tar-bound invariants.
 *        Full-sort comparison and copy counts: parity unpinned (the paper prints
 *        them only in figures that are not part of its text, and the readings
 *        of the unprinted pivot code change them).
 *   oracle_median3_i32   pinned: exact comparisons, copies, result and flag for
 *        all 13 weak orderings of three keys, traced by hand from the listing of
 *        SIII.I (tests/golden/median3_counts.txt).
 *   oracle_insertion_i32 pinned: comparisons and copies equal the closed form
 *        in the inversion table that the SIV listing implies.
 *   oracle_median5_i32   pinned: for every permutation and every weak ordering
 *        of five keys, the samples end sorted in place, the pivot is the third
 *        smallest and the flag follows the order of the input.  Its comparison
 *        and copy counts: parity unpinned (the paper's generated tree is not
 *        printed, reading R4).
 *   oracle_choose_pivot_i32  pinned: sample positions of the ninther and the
 *        fifteenther worked out by hand (with and without the jitter of SV.C)
 *        on arrays that hold distinct values only there; the pivot is the
 *        median of the medians and the flag follows reading R5.
 *   oracle_run_entry_i32 pinned: hand-traced entry states of States 2L/2R,
 *        3L/3R and exit2 (tests/golden/stage_traces.txt).
 */
#include "tsqs_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ---- the total orders (three-valued, as the paper's cmp, SIII) ---------- */

static inline int ord_i32(int32_t x, int32_t y) { return (x > y) - (x < y); }
static inline int ord_u32(uint32_t x, uint32_t y) { return (x > y) - (x < y); }
static inline int ord_i64(int64_t x, int64_t y) { return (x > y) - (x < y); }
static inline int ord_u64(uint64_t x, uint64_t y) { return (x > y) - (x < y); }

/* IEEE 754-2008 totalOrder (clause 5.10) on binary32 bit patterns:
 * -NaN < -inf < negative finite < -0 < +0 < positive finite < +inf < +NaN,
 * NaNs ordered by payload; identical bits compare equal and nothing else does.
 * By cases on the sign bits: a negative value is below a positive one; two
 * positives order as their magnitude bits; two negatives in reverse. */
static inline int ord_f32bits(uint32_t x, uint32_t y) {
  uint32_t sx = x >> 31, sy = y >> 31;
  uint32_t mx = x & 0x7FFFFFFFu, my = y & 0x7FFFFFFFu;
  if (sx != sy) return sx ? -1 : 1;
  if (!sx) return (mx > my) - (mx < my);
  return (mx < my) - (mx > my);
}

typedef struct { int32_t k; uint32_t v; } pr_i32;
typedef struct { uint32_t k; uint32_t v; } pr_u32;
typedef struct { int64_t k; uint32_t v; } pr_i64;
typedef struct { uint64_t k; uint32_t v; } pr_u64;
typedef struct { uint32_t k; uint32_t v; } pr_f32;

/* ---- instantiations ----------------------------------------------------- */

#define ELEM int32_t
#define KCMP(x, y) ord_i32((x), (y))
#define SFX i32
#define HAS_ID 0
#include "tsqs_stage.inc"
#undef ELEM
#undef KCMP
#undef SFX
#undef HAS_ID
#undef FN
#undef CAT_
#undef CAT2_

#define ELEM uint32_t
#define KCMP(x, y) ord_u32((x), (y))
#define SFX u32
#define HAS_ID 0
#include "tsqs_stage.inc"
#undef ELEM
#undef KCMP
#undef SFX
#undef HAS_ID
#undef FN
#undef CAT_
#undef CAT2_

#define ELEM int64_t
#define KCMP(x, y) ord_i64((x), (y))
#define SFX i64
#define HAS_ID 0
#include "tsqs_stage.inc"
#undef ELEM
#undef KCMP
#undef SFX
#undef HAS_ID
#undef FN
#undef CAT_
#undef CAT2_

#define ELEM uint64_t
#define KCMP(x, y) ord_u64((x), (y))
#define SFX u64
#define HAS_ID 0
#include "tsqs_stage.inc"
#undef ELEM
#undef KCMP
#undef SFX
#undef HAS_ID
#undef FN
#undef CAT_
#undef CAT2_

#define ELEM uint32_t
#define KCMP(x, y) ord_f32bits((x), (y))
#define SFX f32
#define HAS_ID 0
#include "tsqs_stage.inc"
#undef ELEM
#undef KCMP
#undef SFX
#undef HAS_ID
#undef FN
#undef CAT_
#undef CAT2_

#define ELEM pr_i32
#define KCMP(x, y) ord_i32((x).k, (y).k)
#define SFX pi32
#define HAS_ID 1
#include "tsqs_stage.inc"
#undef ELEM
#undef KCMP
#undef SFX
#undef HAS_ID
#undef FN
#undef CAT_
#undef CAT2_

#define ELEM pr_u32
#define KCMP(x, y) ord_u32((x).k, (y).k)
#define SFX pu32
#define HAS_ID 1
#include "tsqs_stage.inc"
#undef ELEM
#undef KCMP
#undef SFX
#undef HAS_ID
#undef FN
#undef CAT_
#undef CAT2_

#define ELEM pr_i64
#define KCMP(x, y) ord_i64((x).k, (y).k)
#define SFX pi64
#define HAS_ID 1
#include "tsqs_stage.inc"
#undef ELEM
#undef KCMP
#undef SFX
#undef HAS_ID
#undef FN
#undef CAT_
#undef CAT2_

#define ELEM pr_u64
#define KCMP(x, y) ord_u64((x).k, (y).k)
#define SFX pu64
#define HAS_ID 1
#include "tsqs_stage.inc"
#undef ELEM
#undef KCMP
#undef SFX
#undef HAS_ID
#undef FN
#undef CAT_
#undef CAT2_

#define ELEM pr_f32
#define KCMP(x, y) ord_f32bits((x).k, (y).k)
#define SFX pf32
#define HAS_ID 1
#include "tsqs_stage.inc"
#undef ELEM
#undef KCMP
#undef SFX
#undef HAS_ID
#undef FN
#undef CAT_
#undef CAT2_

/* ---- parameters ----------------------------------------------------------- */

void oracle_default_params(oracle_params_t *q) {
  memset(q, 0, sizeof *q);
  /* Reading of SIII.H: only "median of 3 below 70" is printed (SV.C); the
   * other tier bounds are this oracle's defaults. */
  q->ins_max = 12;
  q->med3_below = 70;
  q->med5_below = 800;
  q->ninther_below = 30000;
  q->medof3_small = 1;
  q->random_samples = 1;
  q->handlers = 1;
  q->reverse_tolerance = 3;   /* REVERSE_TOLERANCE is not printed */
  q->analysis_random_pivot = 0;
  q->debug_checks = 0;
  q->seed = 12345u;
}

/* Every tier must get enough elements for distinct sample positions. */
static int params_ok(const oracle_params_t *q) {
  int32_t lo;
  if (q->ins_max < 2) return 0;
  if (q->reverse_tolerance < 0) return 0;
  if (q->analysis_random_pivot) return q->ins_max == 2;
  lo = q->ins_max + 1;                         /* smallest part that is partitioned */
  if (q->medof3_small && q->med3_below > lo) lo = q->med3_below;
  if (lo < q->med5_below && lo < 5) return 0;  /* median of 5 needs n' >= 5 */
  if (q->med5_below > lo) lo = q->med5_below;
  if (lo < q->ninther_below && lo < 9) return 0;
  if (q->ninther_below > lo) lo = q->ninther_below;
  if (lo < 15) return 0;                       /* fifteenther needs n' >= 15 */
  return 1;
}

void oracle_free_storage(void) {
  free_store_i32(); free_store_u32(); free_store_i64(); free_store_u64(); free_store_f32();
  free_store_pi32(); free_store_pu32(); free_store_pi64(); free_store_pu64(); free_store_pf32();
}

/* ---- exported sorts ------------------------------------------------------- */

#define KEYS_ONLY(SUF, T)                                                          \
  int oracle_tsqs_sort_##SUF(T *keys, size_t n, const oracle_params_t *prm,       \
                             oracle_counters_t *cnt) {                             \
    oracle_params_t dp;                                                            \
    oracle_counters_t dc;                                                          \
    if (!prm) { oracle_default_params(&dp); prm = &dp; }                           \
    if (!cnt) cnt = &dc;                                                           \
    memset(cnt, 0, sizeof *cnt);                                                   \
    if (!params_ok(prm)) return -1;                                                \
    if (n > 1 && !keys) return -1;                                                 \
    return sort_elems_##SUF(keys, n, prm, cnt);                                    \
  }

KEYS_ONLY(i32, int32_t)
KEYS_ONLY(u32, uint32_t)
KEYS_ONLY(i64, int64_t)
KEYS_ONLY(u64, uint64_t)
KEYS_ONLY(f32, uint32_t)

#define PAIRS(SUF, PSUF, T, PT)                                                     \
  int oracle_tsqs_sort_pairs_##SUF(T *keys, uint32_t *vals, size_t n,               \
                                   const oracle_params_t *prm,                       \
                                   oracle_counters_t *cnt) {                         \
    oracle_params_t dp;                                                              \
    oracle_counters_t dc;                                                            \
    PT *e;                                                                           \
    size_t i;                                                                        \
    int rc;                                                                          \
    if (!prm) { oracle_default_params(&dp); prm = &dp; }                             \
    if (!cnt) cnt = &dc;                                                             \
    memset(cnt, 0, sizeof *cnt);                                                     \
    if (!params_ok(prm)) return -1;                                                  \
    if (n < 2) return 0;                                                             \
    if (!keys || !vals) return -1;                                                   \
    e = (PT *)malloc(n * sizeof(PT));                                                \
    if (!e) return -3;                                                               \
    for (i = 0; i < n; i++) { e[i].k = keys[i]; e[i].v = vals[i]; }                  \
    rc = sort_elems_##PSUF(e, n, prm, cnt);                                          \
    for (i = 0; i < n; i++) { keys[i] = e[i].k; vals[i] = e[i].v; }                  \
    free(e);                                                                         \
    return rc;                                                                       \
  }

PAIRS(i32, pi32, int32_t, pr_i32)
PAIRS(u32, pu32, uint32_t, pr_u32)
PAIRS(i64, pi64, int64_t, pr_i64)
PAIRS(u64, pu64, uint64_t, pr_u64)
PAIRS(f32, pf32, uint32_t, pr_f32)

/* ---- test hooks ------------------------------------------------------------ */

int oracle_median3_i32(int32_t *ar3, int32_t *piv, oracle_counters_t *cnt) {
  ctx_i32 c;
  oracle_params_t q;
  int flag;
  oracle_default_params(&q);
  memset(&c, 0, sizeof c);
  memset(cnt, 0, sizeof *cnt);
  c.ar = ar3;
  c.prm = &q;
  c.cnt = cnt;
  c.n = 3;
  flag = median3_i32(&c, 0, 1, 2, 1);
  *piv = c.p;
  return flag;
}

int oracle_insertion_i32(int32_t *ar, size_t n, oracle_counters_t *cnt) {
  ctx_i32 c;
  oracle_params_t q;
  oracle_default_params(&q);
  memset(&c, 0, sizeof c);
  memset(cnt, 0, sizeof *cnt);
  if (n < 2) return 0;
  c.ar = ar;
  c.prm = &q;
  c.cnt = cnt;
  c.n = n;
  insertion_i32(&c, 0, (ptrdiff_t)n - 1);
  return 0;
}

int oracle_median5_i32(int32_t *ar5, int32_t *piv, oracle_counters_t *cnt) {
  ctx_i32 c;
  oracle_params_t q;
  ptrdiff_t pos[5] = {0, 1, 2, 3, 4};
  int flag;
  oracle_default_params(&q);
  memset(&c, 0, sizeof c);
  memset(cnt, 0, sizeof *cnt);
  c.ar = ar5;
  c.prm = &q;
  c.cnt = cnt;
  c.n = 5;
  flag = median5_i32(&c, pos, 1);
  *piv = c.p;
  return flag;
}

int oracle_choose_pivot_i32(int32_t *ar, size_t n, const oracle_params_t *prm, int32_t *piv,
                            oracle_counters_t *cnt) {
  ctx_i32 c;
  int flag;
  memset(&c, 0, sizeof c);
  memset(cnt, 0, sizeof *cnt);
  if (!ar || !prm || n < 3) return -2;
  c.ar = ar;
  c.prm = prm;
  c.cnt = cnt;
  c.n = n;
  c.zgen = prm->seed & 0x7FFFFFFFu;
  if (c.zgen == 0) c.zgen = 1;
  c.zgen = pm_step_i32(c.zgen);
  c.dran = 0.5 + (double)c.zgen / 2147483648.0;
  flag = choose_pivot_i32(&c, 0, (ptrdiff_t)n - 1, ((ptrdiff_t)n - 1) >> 1);
  *piv = c.p;
  return flag;
}

int oracle_run_entry_i32(int32_t *ar, size_t n, oracle_entry_t *e, oracle_counters_t *cnt) {
  ctx_i32 c;
  frm_i32 f;
  oracle_params_t q;
  int32_t *tar;
  int rc = 0;
  memset(cnt, 0, sizeof *cnt);
  if (!ar || !e || n < 2 || e->a < 0 || e->b >= (int64_t)n || e->a > e->b) return -1;
  oracle_default_params(&q);
  memset(&c, 0, sizeof c);
  tar = (int32_t *)malloc((n / 2 + 1) * sizeof(int32_t));
  c.hole = (unsigned char *)calloc(n, 1);
  if (!tar || !c.hole) { free(tar); free(c.hole); return -3; }
  c.ar = ar;
  c.tar = tar;
  c.tar_cap = (ptrdiff_t)(n / 2 + 1);
  c.prm = &q;
  c.cnt = cnt;
  c.n = n;
  c.p = e->p;
  c.temp = e->temp;
  c.hole[e->hole0] = 1;
  c.hole[e->hole1] = 1;
  f.a = e->a; f.b = e->b; f.mid = e->a + ((e->b - e->a) >> 1);
  f.l = e->l; f.r = e->r; f.m = e->m; f.ml = e->ml; f.mr = e->mr;
  f.lc = e->lc;
  f.pivot_at_mid = 0;
  c.lo = e->a; c.hi = e->b;
  c.budget = 64 * (int64_t)(e->b - e->a + 1) + 256;
  if (setjmp(c.bail)) {
    rc = -2;
  } else {
    c.armed = 1;
    if (e->entry == OR_STATE2) state2_i32(&c, &f, e->open_side ? HI : LO);
    else if (e->entry == OR_STATE3) state3_i32(&c, &f, e->open_side ? HI : LO);
    if (e->entry == OR_STATE2 || e->entry == OR_STATE3 || e->entry == OR_EXIT2) exit2_i32(&c, &f);
    else rc = -1;
    c.armed = 0;
  }
  e->l = f.l; e->r = f.r; e->m = f.m; e->ml = f.ml; e->mr = f.mr;
  for (int64_t x = 0; x < (int64_t)n; x++) if (c.hole[x]) cnt->hole_errors++;
  free(tar);
  free(c.hole);
  return rc;
}
