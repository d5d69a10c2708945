/*
 * tsqs.h -- C ABI of libtsqs, a three-way partition sort for AMD MI355X (gfx950).
 *
 * The operation is the one of Triple State QuickSort (Muqaddas, arXiv
 * 1505.00558): sort nmemb elements in ascending order, in place, qsort-style
 * (abstract and SVII of the paper), by recursive partitioning around a sampled
 * pivot where every key equal to the pivot is put in a middle band and never
 * compared again (SIII, the "equals partition").  Here the elements are
 * fixed-width keys resident in device memory, optionally carrying a uint32
 * payload; the order is compiled in:
 *   int32 / int64 / uint32 / uint64  the usual integer order;
 *   float32                          IEEE 754-2008 totalOrder on the bits:
 *       -NaN < -inf < -finite < -0.0 < +0.0 < +finite < +inf < +NaN,
 *       NaNs ordered by payload; two keys are equal iff their bits are equal.
 * Output keys are therefore unique (the sorted arrangement of the input
 * multiset).  Payload order among equal keys is unspecified (the sort is not
 * stable), but every payload stays with its key.
 *
 * Ownership.  The caller owns the key / payload buffers (device memory, e.g.
 * a hipMalloc'd pointer or a torch tensor's data_ptr()).  The library owns a
 * per-device workspace (a scratch copy of the keys and payloads plus small
 * tables) that grows to the largest request seen and is kept between calls,
 * as the paper keeps its temporary buffer (SIII.G); tsqs_free_storage()
 * releases it (the paper's FreeTripleStateQuickSortStorage()).
 *
 * Streams and synchronisation.  All work is enqueued on `stream` (a
 * hipStream_t; NULL = the default stream) and the call returns without waiting
 * for it: the caller synchronises (the stream, or an event recorded after the
 * call) before it reads the buffers.  The schedule needs no answer from the
 * device: the levels a median split needs are launched, and one persistent
 * kernel finishes whatever they leave (bad pivots, the depth-limit fallback).
 * Calls are serialised by a library mutex; a call on another stream than the
 * previous one waits (on the device) for the previous one, since they share
 * the workspace.
 *
 * Errors.  Argument errors are returned before any HIP call is made.  A HIP
 * runtime failure returns TSQS_EDEVICE; a workspace allocation failure
 * TSQS_ENOMEM.  An error found on the device (an internal capacity or count
 * violation, the persistent kernel's iteration cap) is returned by
 * tsqs_get_stats for that call (TSQS_EINTERNAL).  In every error case the
 * contents of the caller's buffers are unspecified.
 */
#ifndef TSQS_H
#define TSQS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TSQS_INT32 = 0,
  TSQS_UINT32 = 1,
  TSQS_INT64 = 2,
  TSQS_UINT64 = 3,
  TSQS_FLOAT32 = 4
} tsqs_dtype_t;

enum {
  TSQS_OK = 0,
  TSQS_EINVAL = -1,        /* bad pointer, size or offsets */
  TSQS_ENOMEM = -2,        /* workspace could not be allocated */
  TSQS_EDEVICE = -3,       /* HIP runtime error */
  TSQS_EUNSUPPORTED = -4,  /* unknown dtype or option */
  TSQS_EINTERNAL = -5,     /* capacity / level limit exceeded (a bug) */
  TSQS_ESCRATCH = -7       /* tsqs_sort_noalloc: the request does not fit its fixed scratch */
};

/* Option keys for tsqs_set_option / tsqs_get_option. */
enum {
  TSQS_OPT_SMALL_MAX = 1,    /* parts of at most this many keys are finished by
                                one workgroup in LDS (paper SIV's cutoff role);
                                16..8192 (4096 for 64-bit keys with payload) */
  TSQS_OPT_SAMPLES = 2,      /* pivot samples per part, odd, 3..63 (SIII.H) */
  TSQS_OPT_DEPTH_FACTOR = 3, /* depth limit = factor * ceil(log2 n); a part at the
                                limit gets the exact median (introsort idea, SV.C) */
  TSQS_OPT_PIVOT_MODE = 4,   /* 0 = median of samples; 1 = exact minimum (test
                                knob that forces the depth-limit fallback) */
  TSQS_OPT_SEED = 5,         /* seed of the per-call sample jitter (SV.C) */
  TSQS_OPT_TIMING = 6,       /* 1 = time every partition launch with HIP events */
  TSQS_OPT_PART_GRID = 7,    /* workgroups of the partition kernels (0 = auto: 4 per CU;
                                for the two-level kernel over 4-byte keys without
                                payload, as many as are resident at once, 7 per CU) */
  TSQS_OPT_FINISH_GRID = 8,  /* workgroups of the finish kernel (0 = auto: 32 per CU) */
  TSQS_OPT_FINISH_ALGO = 9,  /* small parts: 0 = bitonic sorting network, 1 = per-thread
                                sorting network + merge-path merging in LDS, one output
                                at a time, 3 = runs of up to one wave merged by
                                cross-lane bitonic stages in registers first, then as 1
                                (default), 2 = as 3 with each thread's outputs of a
                                merge in LDS merged by a register network */
  TSQS_OPT_PRESORT = 10,     /* 1 (default) = before the first pass of an array that
                                needs one (tsqs_sort, tsqs_sort_pairs, each array of
                                tsqs_sort_batch), check whether it is already
                                non-decreasing, or non-increasing (then reverse it in
                                place, payloads too): such an array needs no pass (the
                                sorted / reversed handlers, SIII.I); 0 = off.  The
                                serving queue does not check */
  TSQS_OPT_SCHEDULE = 11,    /* 0 (default) = the level schedule (one to three kernels
                                per recursion level, the levels a median split needs),
                                then the persistent kernel for what is left; 1 = the
                                persistent kernel for every part (one launch after the
                                roots are set up) */
  TSQS_OPT_ITER_CAP = 12,    /* loop iterations (tasks and waits) of one workgroup of
                                the persistent kernel before it stops every workgroup
                                and reports an error; 0 (default) = 2^23 (a wait of
                                some seconds; a run of the kernel takes far fewer) */
  TSQS_OPT_QUEUE_DIRECT = 13, /* serving queues opened after this: requests of at
                                least this many keys are sorted by the single-array
                                schedule on a stream of the queue's own instead of
                                the queue's ticks (tsqs_queue.h); 0 = never;
                                default 2^22 */
  TSQS_OPT_PART_THREADS1 = 14, /* workgroup size of the one-level partition kernel: 512
                                (default; 32 4-byte keys per thread) or 1024 (16 per
                                thread); a chunk is the same 16384 keys either way */
  TSQS_OPT_PART_THREADS2 = 15, /* workgroup size of the two-level partition kernel: 256
                                (default; 32 4-byte keys per thread) or 512 (16 per
                                thread); a chunk is the same 8192 keys either way */
  TSQS_OPT_WORKSPACE_CAP = 16, /* bytes the per-device workspace of the sort calls may
                                hold (0 = no cap, the default); a call that would grow
                                it past the cap returns TSQS_ENOMEM before it allocates,
                                frees or launches anything (the keys are untouched) */
  TSQS_OPT_DEBUG = 17        /* 1 = debug shadows for tsqs_sort / _pairs / _batch /
                                _records and graphs created while on (3 n words more
                                workspace, no presortedness check): every store of a
                                partition pass is checked to land on a slot that no
                                other key of the same part's pass took (the chunk
                                reservations are disjoint) and that is not final; every
                                slot of the keys receives its final key exactly once (a
                                band or a small part), and all of them do.  A violation
                                sets TSQS_ERR_SHADOW in tsqs_stats_t.error_flags
                                (tsqs_get_stats returns TSQS_EINTERNAL).  0 = off
                                (default).  2 and 3 are test modes of the checks: as
                                1, with one shadow entry planted before the sort (slot
                                0 of the keys already final / slot 0 of the scratch
                                copy already stored by the root's pass), so that a
                                correct sort reports TSQS_ERR_SHADOW */
};

#define TSQS_MAX_LEVELS 192

typedef struct {
  uint32_t levels;               /* partition levels launched */
  uint32_t max_depth;            /* deepest partitioned part */
  uint64_t n;                    /* keys sorted */
  uint32_t key_bytes;            /* 4 or 8 */
  uint32_t payload_bytes;        /* 0 or 4 */
  uint64_t fallback_parts;       /* parts that got the exact median */
  uint64_t small_parts;          /* parts finished in LDS */
  uint64_t small_keys;           /* keys finished in LDS */
  uint64_t band_keys;            /* keys placed by an equal band */
  uint64_t level_keys[TSQS_MAX_LEVELS];     /* keys partitioned at each level */
  uint32_t level_parts[TSQS_MAX_LEVELS];    /* parts partitioned at each level */
  float level_ms[TSQS_MAX_LEVELS];          /* partition kernel time (TIMING) */
  double partition_ms;           /* sum of level_ms */
  uint64_t partition_bytes;      /* algorithmic bytes: 2 * keys * (key+payload bytes) */
  uint32_t partition_launches;   /* partition kernel launches (one per level with parts) */
  uint32_t presorted;            /* single array: 0; 1 = found non-decreasing, 2 = found
                                    non-increasing and reversed (TSQS_OPT_PRESORT): no pass
                                    was needed.  Batch: arrays found in order */
  uint64_t tail_parts;           /* parts partitioned by the persistent kernel */
  uint64_t tail_keys;            /* keys of those parts */
  uint64_t tail_bytes;           /* their algorithmic bytes, 2 * keys * (key+payload bytes) */
  uint64_t select_rounds;        /* radix digits fixed by grid-wide exact-pivot selection */
  uint32_t error_flags;          /* device error bits of the call (0 = none; TSQS_ERR_*) */
  uint32_t schedule;             /* TSQS_OPT_SCHEDULE of the call */
} tsqs_stats_t;

/* Bits of tsqs_stats_t.error_flags. */
#define TSQS_ERR_SEG_CAP 1u     /* a level's part table was full */
#define TSQS_ERR_FIN_CAP 2u     /* a small-part or band table was full */
#define TSQS_ERR_LEVEL 4u       /* more levels than the level table holds */
#define TSQS_ERR_COUNT 8u       /* class counts that do not fit their part */
#define TSQS_ERR_QUEUE 16u      /* persistent schedule: task ring or part pool full */
#define TSQS_ERR_ITER 32u       /* persistent schedule: iteration cap reached */
#define TSQS_ERR_SHADOW 128u    /* TSQS_OPT_DEBUG: a shadow check failed */

/* Sort nmemb keys of type dt at device pointer d_keys, in place (the paper's
 * problem statement, abstract and SVII).  nmemb <= 1 is a no-op.  nmemb must
 * be < 2^32 (part lengths and the packed left|right cursor reservation of the
 * partition pass are 32-bit).  Returns TSQS_OK or an error code. */
int tsqs_sort(void *d_keys, size_t nmemb, int dt, void *stream);

/* As tsqs_sort, moving the uint32 payload d_vals[i] with key d_keys[i]. */
int tsqs_sort_pairs(void *d_keys, uint32_t *d_vals, size_t nmemb, int dt, void *stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): as
 * tsqs_sort (d_vals NULL) or tsqs_sort_pairs, but every device buffer of the
 * call -- the scratch copy of the keys and payloads, the level tables, the
 * small-part and band slots, the statistics -- is taken from one fixed array
 * of TSQS_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends.  The call makes no hipMalloc, hipFree or other
 * allocation.
 *   nmemb <= TSQS_NOALLOC_MAX_KEYS; a larger request, or one whose buffers
 *   for the current options (a small TSQS_OPT_SMALL_MAX needs more tables)
 *   exceed the array, returns TSQS_ESCRATCH before any device work.
 * Every call on a GPU uses that GPU's one array and leaves its contents
 * behind (what must start at zero is cleared by the call's first kernel):
 * calls whose device work overlaps on one GPU race; the caller orders them
 * (one stream, or events).  Other conventions as tsqs_sort. */
#define TSQS_NOALLOC_MAX_KEYS (1u << 20)
#define TSQS_NOALLOC_SCRATCH_BYTES (32u << 20)
int tsqs_sort_noalloc(void *d_keys, uint32_t *d_vals, size_t nmemb, int dt, void *stream);

/* Sort records of any size by their keys (late swapping, SVIII.H): the keys
 * are sorted in place with a uint32 index as their payload (the paper's
 * temporary pointer array), then every record is moved once, by a gather,
 * into its sorted place.
 *   d_keys     nmemb keys of type dt (device), sorted in place
 *   d_records  nmemb records of rec_bytes bytes each (device), record i
 *              belonging to key i; 1 <= rec_bytes <= 65536
 *   d_out      device buffer for the records in key order (d_records is then
 *              left as it was; the two must not overlap), or NULL (or
 *              d_records) to reorder d_records in place through a staging
 *              buffer of nmemb * rec_bytes bytes that the library allocates and
 *              keeps (freed by tsqs_free_storage)
 * nmemb < 2^32.  Records with equal keys come out in no particular order.
 * Returns TSQS_EINVAL for null pointers, bad sizes or overlapping buffers;
 * TSQS_EINTERNAL if the sorted index was not a permutation (a bug). */
int tsqs_sort_records(void *d_keys, void *d_records, size_t rec_bytes, void *d_out, size_t nmemb,
                      int dt, void *stream);

/* Sort nseg independent arrays stored back to back in d_keys: array j is
 * d_keys[h_offsets[j] .. h_offsets[j+1]).  The paper measures the overhead of
 * many small sorts (SIX); here every array's parts of a level share the same
 * launches (or the one persistent kernel, TSQS_OPT_SCHEDULE 1), so the cost
 * per array is not a launch.  h_offsets is a host array of nseg+1
 * non-decreasing values starting at 0 (copied during the call); every array
 * must have < 2^32 keys (the total may exceed that).  d_vals may be NULL
 * (keys only) or a payload array of the same layout. */
int tsqs_sort_batch(void *d_keys, uint32_t *d_vals, const uint64_t *h_offsets, size_t nseg,
                    int dt, void *stream);

/* Result of tsqs_autotune: the options it chose and the times it measured. */
typedef struct {
  int64_t small_max;     /* TSQS_OPT_SMALL_MAX */
  int64_t samples;       /* TSQS_OPT_SAMPLES */
  int64_t part_grid;     /* TSQS_OPT_PART_GRID (workgroups) */
  int64_t finish_grid;   /* TSQS_OPT_FINISH_GRID (workgroups) */
  int64_t finish_algo;   /* TSQS_OPT_FINISH_ALGO */
  double ms_default;     /* sort time with the options in force at the call */
  double ms_best;        /* sort time with the chosen options */
  uint32_t trials;       /* configurations timed (0: taken from the tuning cache) */
  uint32_t reserved;
  int64_t part_threads1; /* TSQS_OPT_PART_THREADS1 */
  int64_t part_threads2; /* TSQS_OPT_PART_THREADS2 */
} tsqs_tune_t;

/* Autotuner: times sorts of seeded uniform keys of type dt (with a uint32
 * payload if with_payload) shaped like the caller's work -- one array of n keys
 * when h_offsets is NULL, else the nseg arrays of h_offsets (as for
 * tsqs_sort_batch; n must equal h_offsets[nseg]) -- over candidate values of
 * the small-part threshold, the pivot sample count, the partition and finish
 * grids, the small-part algorithm and the partition kernels' workgroup sizes
 * (threads against keys per thread; one parameter at a time, keeping the best
 * so far), then sets the fastest as the current options and reports it in *out
 * (may be NULL).  Uses 2 n keys (+ 2 n payloads) of temporary device memory,
 * freed before it returns.  Returns TSQS_OK or an error code; on error the
 * options in force at the call are restored.
 *
 * Tuning cache: when the environment variable TSQS_TUNE_CACHE names a file, a
 * line there for the same device architecture (gcnArchName up to its first
 * ':'), key type, payload, batch or single array, and ceil(log2 n) is applied
 * without timing anything (out->trials = 0); otherwise the tuner runs and
 * appends its result as one text line.  The file is read and appended under
 * the library's lock, so the threads of one process share it; separate
 * processes must not tune into the same file at the same time. */
int tsqs_autotune(int dt, int with_payload, size_t n, const uint64_t *h_offsets, size_t nseg,
                  void *stream, tsqs_tune_t *out);

/* Graphs, for callers that sort the same buffers, of the same shape, many
 * times (a batch of fixed array sizes refilled between sorts, a serving slot):
 * the whole schedule of one call is captured once into a HIP graph and then
 * replayed with one launch.  The operation of a replay is that of tsqs_sort /
 * tsqs_sort_batch (the paper's problem statement, abstract and SVII; the
 * repeated calls of SIX's overhead tests); the graph itself has no paper
 * counterpart. 
 *
 * tsqs_graph_create captures the sort of nmemb keys at d_keys (and payloads at
 * d_vals, or NULL): one array when h_offsets is NULL, else the nseg arrays of
 * h_offsets, with h_offsets[nseg] == nmemb (as tsqs_sort_batch; the offsets are
 * copied to the device at creation and not read again).  Argument rules and
 * limits are those of tsqs_sort / tsqs_sort_pairs / tsqs_sort_batch; a call
 * with nothing to sort (fewer than two keys in every array) returns
 * TSQS_EINVAL.  The options in force at creation are the graph's.  The graph
 * owns a workspace of its own (about the size tsqs_sort would use), allocated
 * at creation, so other calls of the library neither reuse nor regrow it.
 * Creation waits for the device once (the buffers' first clears); it does not
 * sort.
 *
 * tsqs_graph_launch enqueues one replay on stream (a hipStream_t, NULL = the
 * default stream): it sorts whatever d_keys (and d_vals) hold when the replay
 * runs, like the captured call.  Replays of one graph on different streams are
 * ordered (a launch on another stream waits for the previous launch).
 * tsqs_graph_stats waits for the last launch and reports it like
 * tsqs_get_stats (without per-level times).  tsqs_graph_destroy waits for the
 * last launch and frees the graph. */
typedef struct tsqs_graph tsqs_graph_t;
int tsqs_graph_create(void *d_keys, uint32_t *d_vals, size_t nmemb, const uint64_t *h_offsets,
                      size_t nseg, int dt, tsqs_graph_t **out);
int tsqs_graph_launch(tsqs_graph_t *g, void *stream);
int tsqs_graph_stats(tsqs_graph_t *g, tsqs_stats_t *out);
int tsqs_graph_destroy(tsqs_graph_t *g);

/* Release the workspace of every device (SIII.G's manual release). */
void tsqs_free_storage(void);

int tsqs_set_option(int key, int64_t value);
/* Returns the option's value, or INT64_MIN for an unknown key. */
int64_t tsqs_get_option(int key);

/* Statistics of the last call: passes and keys per level, fallbacks, keys
 * finished in LDS or by bands, the persistent kernel's share -- the GPU
 * counterparts of the paper's comparison and copy counts (SV.A, SVI).  Waits
 * for the call's device work; returns TSQS_EINTERNAL (with *out filled) if the
 * device reported an error for it, TSQS_EINVAL if there was no call. */
int tsqs_get_stats(tsqs_stats_t *out);

const char *tsqs_strerror(int code);

/* ABI version (increments when this header changes incompatibly). */
int tsqs_version(void);

#ifdef __cplusplus
}
#endif
#endif
