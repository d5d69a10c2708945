/*
 * tsqs_queue.h -- serving queue of libtsqs: many independent sort requests,
 * continuously batched on one device.
 *
 * The paper's operation is a single qsort-shaped call (sort nmemb elements
 * ascending, SVII); this interface serves a stream of such calls.  Requests are
 * copied into a device arena held within an HBM budget, and each "tick"
 * advances every live request of a key type by one level of the three-way
 * partition recursion (SIII): one partition pass over all their current parts,
 * the pivot / child planning, and the finishing of small parts and equal bands.
 * Requests admitted at a tick join that tick's launches, so a new request's
 * first levels run in the same kernels as older requests' deeper levels.
 * Results stay in the arena (sorted in place there) until released.
 *
 * Large requests.  A request of at least TSQS_OPT_QUEUE_DIRECT keys (the value
 * when the queue was opened; default 2^22, 0 = none) does not join the ticks:
 * its keys are copied into the arena and sorted there by the single-array
 * schedule of tsqs_sort, on a stream of the queue's own, one such request after
 * another.  Such a sort already runs at the single-array rate, and it does not
 * wait a tick per recursion level.  These sorts use the library's per-device
 * workspace, which tsqs_sort also uses: calls on other streams are ordered
 * after them, and tsqs_get_stats keeps reporting the caller's own last call.
 *
 * Ownership.  The queue owns its arena (keys and the scratch copy, each half of
 * the budget less the level tables), its tables and a page of host-mapped
 * completion flags.  The caller owns each request's source buffer, which must
 * stay valid and unchanged until the request has been admitted (state >= 1).
 *
 * Streams.  The queue's device work runs on streams of its own, one per key
 * type (created at the default priority), so ticks of different key types
 * overlap.  Work enqueued on the stream given to tsqs_queue_open before a
 * request is admitted completes before the queue reads that request's source.
 * tsqs_queue_step does not wait for the device (a key type whose ticks in
 * flight are at their limit is skipped until one finishes), except when a large
 * request needs a larger workspace than any call before it: the workspace is
 * regrown after the work that uses it.  tsqs_queue_poll and tsqs_queue_reap
 * read host-mapped memory and event states and never wait.  A queue is used from
 * one host thread at a time (calls are serialised by a per-queue mutex).
 *
 * Errors are the TSQS_* codes of tsqs.h; TSQS_EAGAIN (below) means "not yet".
 */
#ifndef TSQS_QUEUE_H
#define TSQS_QUEUE_H

#include <stddef.h>
#include <stdint.h>

#include "tsqs.h"

#ifdef __cplusplus
extern "C" {
#endif

#define TSQS_EAGAIN (-6)   /* the request is not done yet / no room yet */

typedef struct tsqs_queue tsqs_queue_t;

/* Open a queue on the current device.  budget_bytes bounds the device memory
 * of the arena and the tables (at least 64 MiB); stream is a hipStream_t (NULL =
 * the default stream).  On success *out is the queue. */
int tsqs_queue_open(size_t budget_bytes, void *stream, tsqs_queue_t **out);

/* Queue a request: nmemb keys of type dt at device pointer d_src (1 <= nmemb <
 * 2^32).  Returns TSQS_OK and a ticket; TSQS_ENOMEM if the request can never fit
 * the arena.  Admission is first in, first out, as arena space frees up. */
int tsqs_queue_submit(tsqs_queue_t *q, const void *d_src, size_t nmemb, int dt,
                      uint64_t *ticket);

/* Admit what fits (copying the keys into the arena) and launch one tick for
 * every key type with live requests.  Returns TSQS_OK, or an error (a device
 * failure, or TSQS_EINTERNAL if a kernel reported a capacity violation). */
int tsqs_queue_step(tsqs_queue_t *q);

/* State of a request: 0 queued, 1 admitted and running, 2 done (its keys are
 * sorted in the arena), or TSQS_EINVAL for an unknown or released ticket. */
int tsqs_queue_poll(tsqs_queue_t *q, uint64_t ticket);

/* Device pointer and length of a done request's sorted keys (valid until
 * tsqs_queue_release); TSQS_EAGAIN if it is not done. */
int tsqs_queue_result(tsqs_queue_t *q, uint64_t ticket, void **d_keys, size_t *nmemb);

/* Tickets of requests found done since the previous call (at most cap of them,
 * oldest first; the rest are returned by later calls).  *count = number
 * written. */
int tsqs_queue_reap(tsqs_queue_t *q, uint64_t *tickets, size_t cap, size_t *count);

/* Give a done request's arena space back (TSQS_EAGAIN if it is not done). */
int tsqs_queue_release(tsqs_queue_t *q, uint64_t ticket);
/* Cancel a request (serving only; no paper counterpart): one still queued is
 * dropped (never admitted, its source never read), a done one is released; the
 * ticket becomes invalid (TSQS_OK).
 * TSQS_EAGAIN for a running request (its device work is enqueued: release it
 * when done), TSQS_EINVAL for an unknown ticket. */
int tsqs_queue_cancel(tsqs_queue_t *q, uint64_t ticket);

/* Counts: requests queued (not admitted), running, done and not released; arena
 * bytes in use and in total.  Any pointer may be NULL. */
int tsqs_queue_info(tsqs_queue_t *q, uint64_t *queued, uint64_t *running, uint64_t *done,
                    uint64_t *arena_used, uint64_t *arena_bytes);

/* Wait for the device work of the queue, then free it (every ticket becomes
 * invalid). */
int tsqs_queue_close(tsqs_queue_t *q);

#ifdef __cplusplus
}
#endif
#endif
