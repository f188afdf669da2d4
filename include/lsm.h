/*
 * lsm.h -- C ABI of an MI355X (gfx950) batched LSM dictionary.
 *
 * The data structure and its operations are those of Ashkiani, Li,
 * Farach-Colton, Amenta and Owens, "GPU LSM: A Dynamic Dictionary Data
 * Structure for the GPU" (IPDPS 2018, arXiv 1707.05354):
 *
 *   - a dictionary of <key, value> pairs with INSERT, DELETE, LOOKUP, COUNT
 *     and RANGE (sec. I-B), updated in batches of exactly b elements with the
 *     batch semantics of sec. III-A;
 *   - levels of b * 2^i elements, each a sorted array, occupied exactly where
 *     the batch counter r has a set bit; an insertion sorts the batch and
 *     merges it down the full levels like a binary-counter increment
 *     (sec. III-B, Fig. 2(a), Fig. 3);
 *   - deletion as insertion of tombstones (sec. III-C): each stored element
 *     is a 32-bit key variable (original key << 1) | status, status 1 for a
 *     regular element and 0 for a tombstone (sec. IV-A), plus a 32-bit value.
 *
 * Conventions for every call:
 *   - Every array argument whose name starts with d_ is a DEVICE pointer
 *     owned by the caller, on the device the handle was created on.  The
 *     library keeps no caller pointer after the call returns.
 *   - All device work is enqueued on the handle's HIP stream, in call order.
 *     Inputs must stay valid, and outputs are complete, only once that
 *     stream has passed the call (hipStreamSynchronize or an event).  Calls
 *     that must read a result back (lsm_range, checked-mode updates)
 *     synchronise the stream themselves.
 *   - Original keys must be < 2^31 (one bit of the 32-bit key variable holds
 *     the status, sec. IV-A), and < 2^k when the handle was created with
 *     LSM_KEY_BITS(k).  Values are arbitrary 32-bit words.
 *   - Every call returns a status.  On any error the dictionary is left
 *     exactly as it was before the call (strong guarantee).
 *   - A handle is not thread-safe; calls on different handles are
 *     independent, except lsm_range_async_noalloc, whose calls share one
 *     scratch array per GPU (see there).
 */
#ifndef LSM_H_
#define LSM_H_

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define LSM_API __attribute__((visibility("default")))
#else
#define LSM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lsm_s* lsm_t;

typedef enum {
  LSM_OK = 0,
  LSM_EINVAL = 1,    /* null handle or pointer, b out of range, bad flags   */
  LSM_EKEY = 2,      /* checked mode: a key is >= 2^key_bits                */
  LSM_EBATCH = 3,    /* an update batch holds more than b elements          */
  LSM_ENOMEM = 4,    /* a device or pinned-host allocation failed           */
  LSM_ECAPACITY = 5, /* range output larger than cap, or the next level
                        would exceed 2^31 elements                          */
  LSM_EHIP = 6       /* a HIP runtime call or kernel launch failed          */
} lsm_status_t;

/* lsm_create flags. */
#define LSM_CHECKED 0x1u /* validate update keys on the device (syncs)    */
/* Promise that every original key is < 2^k (1 <= k <= 31; default 31).
 * Fewer key bits mean fewer radix-sort passes over each batch. */
#define LSM_KEY_BITS(k) ((((uint32_t)(k)) & 0x3Fu) << 8)

/*
 * lsm_create -- an empty dictionary with batch size b (sec. III-A rule 1:
 * b is fixed and is also the size of level 0).
 *   out    : receives the handle.
 *   b      : batch size, 1 <= b <= 2^28.
 *   flags  : LSM_CHECKED and/or LSM_KEY_BITS(k).
 *   stream : hipStream_t to order all work on (NULL = the default stream);
 *            the device current at this call becomes the handle's device.
 * Allocates the batch scratch (about 40 * b bytes); levels are allocated
 * when an insertion first reaches them.  LSM_EINVAL, LSM_ENOMEM, LSM_EHIP.
 */
LSM_API lsm_status_t lsm_create(lsm_t* out, uint32_t b, uint32_t flags, void* stream);

/* Re-target the handle to another stream of the same device. */
LSM_API lsm_status_t lsm_set_stream(lsm_t h, void* stream);

/*
 * lsm_insert_batch -- INSERT(k, v) for n pairs as one batch (sec. III-B,
 * Fig. 2(a)).  The batch is sorted, then merged down the full levels into
 * the first empty level; the batch counter r grows by one.
 *   d_keys, d_vals : n original keys and n values (device).
 *   n              : 0 <= n <= b.  n == 0 is a no-op (r unchanged).  A batch
 *                    with n < b is padded with copies of its last pair
 *                    (sec. IV-A), so it still occupies b slots.
 * Duplicate keys inside one batch: the last one in batch order wins.
 * Elements staged by lsm_submit / lsm_submit_mixed are older than this batch:
 * when any are pending they are inserted first, as their own padded batch,
 * once everything this batch can be refused for (size, allocations, keys in
 * checked mode) has been checked.
 * LSM_EBATCH if n > b; LSM_EKEY (checked mode); LSM_ENOMEM; LSM_ECAPACITY;
 * LSM_EHIP.
 */
LSM_API lsm_status_t lsm_insert_batch(lsm_t h, const uint32_t* d_keys,
                              const uint32_t* d_vals, uint32_t n);

/*
 * lsm_delete_batch -- DELETE(k) for n keys as one batch: the insertion of
 * n tombstones (sec. III-C), which hide every older instance of their keys.
 * Same size rules and errors as lsm_insert_batch.
 */
LSM_API lsm_status_t lsm_delete_batch(lsm_t h, const uint32_t* d_keys, uint32_t n);

/*
 * lsm_update_batch -- one mixed batch of insertions and deletions
 * (sec. III-A rule 2).  d_is_delete[j] != 0 makes element j a deletion
 * (its value is ignored).  A key inserted and deleted in the same batch
 * ends up deleted (sec. III-A rule 5); otherwise the last insertion of a
 * key in batch order wins.  Same size rules and errors as
 * lsm_insert_batch.
 */
LSM_API lsm_status_t lsm_update_batch(lsm_t h, const uint32_t* d_keys,
                              const uint32_t* d_vals,
                              const uint8_t* d_is_delete, uint32_t n);

/* ---------------------------------------------------------------------
 * Batching form: a coalescer in front of the batch insertion.
 * ------------------------------------------------------------------- */

/*
 * lsm_submit -- one user batch of n >= 0 insertions (is_delete == 0) or
 * deletions (is_delete != 0) of any size.  User batches are packed, in
 * arrival order, into LSM batches of exactly b elements (a user batch may
 * be split across two); every time b elements are staged they are inserted
 * as one batch.  A packed batch means the same as its user batches applied
 * one after another: the newest operation on a key wins whatever its type
 * (unlike lsm_update_batch, where sec. III-A rule 5 makes a key inserted
 * and deleted in one batch deleted).  This implements the partial-batch
 * remark of sec. IV-A (padding costs b'/b of the insertion rate) by packing
 * instead of padding, and the multi-batch ordering of sec. V-B.
 *   d_keys, d_vals : n keys and values (device; d_vals unused for deletes).
 * Staged elements are copied on the stream; the caller's buffers may be
 * reused once the stream has passed the call.  Queries (lsm_lookup,
 * lsm_count, lsm_range) flush the staged elements first.
 * LSM_EKEY (checked mode, nothing staged), LSM_ENOMEM, LSM_ECAPACITY,
 * LSM_EHIP.
 */
LSM_API lsm_status_t lsm_submit(lsm_t h, const uint32_t* d_keys, const uint32_t* d_vals,
                                uint32_t n, int is_delete);

/*
 * lsm_submit_mixed -- stage n operations of both types in arrival order:
 * element j deletes d_keys[j] when d_is_delete[j] != 0 (its value is then
 * ignored) and inserts (d_keys[j], d_vals[j]) otherwise.  One call can carry
 * many user requests; the packing rules of lsm_submit apply, so the newest
 * operation on a key wins whatever its type.  The library encodes each
 * operation as a key variable (sec. IV-A) while staging it.
 *   d_keys, d_vals : n keys and values (device).
 *   d_is_delete    : n flags (device, uint8).
 * Same errors as lsm_submit.
 */
LSM_API lsm_status_t lsm_submit_mixed(lsm_t h, const uint32_t* d_keys, const uint32_t* d_vals,
                                      const uint8_t* d_is_delete, uint32_t n);

/*
 * lsm_flush -- insert the staged elements as one (padded) batch, if any, and
 * enqueue whatever remains of every earlier insertion (an update call may
 * leave the second half of its batch's sort and its cascade to the next
 * update call's launch; queries, cleanup and lsm_sync complete it too).
 * Once the stream has passed the call, every submitted or inserted batch is
 * in the levels.  LSM_ENOMEM, LSM_ECAPACITY, LSM_EHIP.
 */
LSM_API lsm_status_t lsm_flush(lsm_t h);

/* Number of elements staged and not yet inserted. */
LSM_API uint32_t lsm_pending(lsm_t h);

/*
 * Merge-kernel autotuner.  Variant v in [0, 6) merges with 4, 8 or 16
 * elements per thread (v % 3) and at most 1024 or 4096 work-groups (v / 3).
 * lsm_autotune times every variant on merges of two interleaved runs of
 * b * 2^i elements for i = 0 .. max_level (reps launches each, requires
 * b * 2^max_level <= 2^27) and keeps the fastest per level; it synchronises
 * the stream.  lsm_get_tuning returns the chosen variant of merge input
 * level i and, when us != NULL, the 6 measured microseconds per launch.
 */
LSM_API lsm_status_t lsm_autotune(lsm_t h, uint32_t max_level, uint32_t reps);
LSM_API lsm_status_t lsm_get_tuning(lsm_t h, uint32_t level, uint32_t* variant, float* us);
LSM_API lsm_status_t lsm_set_tuning(lsm_t h, uint32_t level, uint32_t variant);

/*
 * lsm_set_fusion -- deepest cascade fused into the top-digit batch sort.  An
 * insert that fills level j <= max_levels (j >= 1) is done by the sort's
 * per-bucket work-groups: each merges its bucket of the batch with the same
 * key range of levels 0..j-1 and writes that part of level j, in the order
 * of the pairwise cascade (so the levels are byte for byte the same), with
 * no merge launch.  0 disables fusion; a negative value restores the
 * default (the largest j with b 2^j <= 2^20, at most 8).  Applies only when
 * the top-digit sort runs.  LSM_EINVAL for more
 * than 8 levels.
 */
LSM_API lsm_status_t lsm_set_fusion(lsm_t h, int max_levels);

/*
 * lsm_set_sort_path -- which batch sort runs (all give the same order, so
 * results never depend on it).  LSM_SORT_TOP_DIGIT: each tile of 2048
 * grouped in place by the top 10 bits of the key variable, then each of the
 * 1024 buckets gathered from every tile and sorted in LDS by one work-group
 * (batches of at most 2^19 elements; larger ones use digit passes).
 * LSM_SORT_DIGIT_PASSES: one stable counting pass
 * per 8-bit digit with decoupled look-back.  LSM_SORT_AUTO (the default):
 * the top-digit sort unless the previous sort saw a top-digit bucket above
 * 1536 elements (skewed keys, where one work-group would sort a large bucket
 * alone).  Takes effect at the next sort.  LSM_EINVAL for another mode.
 */
/*
 * lsm_set_max_inflight -- launch pacing of the update calls.  An update call
 * that sorts its batch by the top-digit sort first waits (spinning on a word
 * of mapped host memory that each such launch writes when it starts, no
 * runtime call) until at most `launches` of its earlier launches are still
 * waiting to start on the stream; 0 turns pacing off.  On MI355X the device
 * ran long queues of these launches markedly slower than short ones, so the
 * default (4) keeps the host a few launches ahead of the device.  A wait
 * gives up after 500 ms.  Results never depend on it.  LSM_EINVAL for a
 * negative value.
 */
LSM_API lsm_status_t lsm_set_max_inflight(lsm_t h, int launches);

/*
 * lsm_set_grouping -- sort consecutive batches together in the top-digit
 * sort: at most max_batches (rounded down to 1, 2 or 4; also capped by b:
 * 4 for b <= 2^17, 2 for b <= 2^18, 1 above; the default is 2 where b
 * allows it).  A
 * batch whose counter r is a multiple of the group size G is held back
 * until the next G - 1 batches have come, and the G batches are then
 * sorted together (the newer first on equal keys) straight into the level
 * the last one fills: one bucket sort for G batches, and the levels below
 * log2 G are never written.  Mixed batches (lsm_update_batch), whose sort
 * orders a key's tombstone before its insertion, never join a group.
 * Queries, cleanup, bulk insertion and lsm_flush complete an incomplete
 * group (as aligned groups of 2 and 1).  max_batches = 1 turns grouping
 * off.  Results never depend on it.  LSM_EINVAL for max_batches < 0.
 */
LSM_API lsm_status_t lsm_set_grouping(lsm_t h, int max_batches);

#define LSM_SORT_AUTO 0
#define LSM_SORT_TOP_DIGIT 1
#define LSM_SORT_DIGIT_PASSES 2
LSM_API lsm_status_t lsm_set_sort_path(lsm_t h, int mode);

/*
 * lsm_lookup -- LOOKUP(k) for nq query keys (sec. III-D, IV-B): searches
 * the occupied levels from the smallest (newest) up; a regular element
 * with key k returns its value, a tombstone with key k ends the search
 * with "not found".
 *   d_keys  : nq query keys (device).
 *   d_vals  : nq outputs; the value, or 0 when not found.
 *   d_found : nq outputs; 1 when found, else 0.
 * nq == 0 is a no-op.  Asynchronous.  LSM_EINVAL, LSM_EHIP.
 */
LSM_API lsm_status_t lsm_lookup(lsm_t h, const uint32_t* d_keys, uint32_t nq,
                        uint32_t* d_vals, uint8_t* d_found);

/*
 * lsm_count -- COUNT(k1, k2) for nq queries (sec. III-E, IV-C): the number
 * of live keys k with d_lo[q] <= k <= d_hi[q] (bounds inclusive; 0 when
 * d_lo[q] > d_hi[q]).  Stale elements and tombstones are not counted.
 *   d_counts : nq outputs (device).
 * nq == 0 is a no-op.  Asynchronous.  LSM_EINVAL, LSM_ENOMEM, LSM_EHIP.
 */
LSM_API lsm_status_t lsm_count(lsm_t h, const uint32_t* d_lo, const uint32_t* d_hi,
                       uint32_t nq, uint32_t* d_counts);

/*
 * lsm_range -- RANGE(k1, k2) for nq queries (sec. III-E, IV-D): every live
 * pair with d_lo[q] <= k <= d_hi[q], per query in ascending key order,
 * queries concatenated in query order.
 *   d_offsets : nq + 1 outputs (device, uint64): the exclusive scan of the
 *               per-query result sizes; d_offsets[nq] is the total.  Always
 *               written.
 *   d_keys, d_vals : outputs of cap elements each (device); written only
 *               when total <= cap.  May be NULL when cap == 0.
 *   cap       : capacity of d_keys / d_vals in elements.
 *   h_total   : HOST pointer; receives the total.
 * Two-phase use: call with cap = 0 to learn the total, allocate, call again.
 * If total > cap the call writes d_offsets and *h_total, writes no keys or
 * values and returns LSM_ECAPACITY.  Synchronises the stream (the total is
 * read back).  LSM_EINVAL, LSM_ENOMEM, LSM_ECAPACITY, LSM_EHIP.
 */
LSM_API lsm_status_t lsm_range(lsm_t h, const uint32_t* d_lo, const uint32_t* d_hi,
                       uint32_t nq, uint64_t* d_offsets, uint32_t* d_keys,
                       uint32_t* d_vals, uint64_t cap, uint64_t* h_total);

/*
 * lsm_bulk_insert -- many insert batches in one call (the bulk build of
 * sec. V-B and its footnote on inserting several batches into a non-empty
 * structure): the n pairs (d_keys[i], d_vals[i]) are exactly ceil(n / b)
 * consecutive insert batches of b elements in array order, the last one
 * partial (padded as lsm_insert_batch pads), so the resulting levels are
 * byte for byte those of the equivalent lsm_insert_batch calls.  Each level
 * of the new batch count that receives new batches is built once: its new
 * batches are sorted together, then merged with the old levels it takes
 * over.  From an empty dictionary this is a sort per level and no merge.
 *   d_keys, d_vals : n keys and values (device), read only.
 * n == 0 is a no-op.  Allocates scratch for the call (the sort's ping-pong
 * and look-back words for the largest level built, two merge buffers when
 * old levels are taken over) and frees it before returning; synchronises
 * the stream.  LSM_EINVAL, LSM_EKEY (checked mode; nothing changed),
 * LSM_ENOMEM (nothing changed), LSM_ECAPACITY (n >= 2^32 or a level above
 * 2^31 elements), LSM_EHIP.
 */
LSM_API lsm_status_t lsm_bulk_insert(lsm_t h, const uint32_t* d_keys, const uint32_t* d_vals,
                                     uint64_t n);

/*
 * lsm_successor / lsm_predecessor -- the order queries that the footnote of
 * sec. I-B names as straightforward extensions: for each of nq query keys,
 * the live pair with the smallest key strictly greater than d_q[i]
 * (successor) or the largest key strictly smaller than d_q[i]
 * (predecessor).  Stale elements and tombstones are skipped exactly as
 * COUNT skips them (sec. III-E).
 *   d_q     : nq query keys (device; any 32-bit value).
 *   d_keys  : nq outputs; the key found, or 0.
 *   d_vals  : nq outputs; its value, or 0.
 *   d_found : nq outputs; 1 when a pair exists, else 0.
 * nq == 0 is a no-op.  Asynchronous.  LSM_EINVAL, LSM_EHIP.
 */
LSM_API lsm_status_t lsm_successor(lsm_t h, const uint32_t* d_q, uint32_t nq,
                                   uint32_t* d_keys, uint32_t* d_vals, uint8_t* d_found);
LSM_API lsm_status_t lsm_predecessor(lsm_t h, const uint32_t* d_q, uint32_t nq,
                                     uint32_t* d_keys, uint32_t* d_vals, uint8_t* d_found);

/*
 * lsm_cleanup -- CLEANUP (sec. III-E) by the bulk strategy of sec. IV-D:
 * removes every tombstone, every deleted element and every replaced
 * duplicate, then rebuilds the levels.  The valid pairs, in ascending key
 * order, are padded with fewer than b placebo elements (tombstones of key
 * 2^31 - 1, which hide nothing) to r' = ceil(valid / b) batches and sliced
 * into the levels of r' from the smallest level up, so smaller keys land in
 * smaller levels.  Every query answer is unchanged; later batches insert on
 * top of r' as usual.
 *   h_valid : HOST pointer (may be NULL); receives the number of valid pairs.
 * Allocates scratch of up to 2 r b (key, value) pairs for the call and frees
 * it before returning; synchronises the stream.  LSM_EINVAL, LSM_ENOMEM
 * (nothing changed), LSM_ECAPACITY (r b >= 2^32), LSM_EHIP.
 */
LSM_API lsm_status_t lsm_cleanup(lsm_t h, uint64_t* h_valid);

/*
 * lsm_clear -- empty the dictionary (r = 0) and keep every allocation, so a
 * rebuild reuses the level memory.  Work already enqueued is unaffected.
 */
LSM_API lsm_status_t lsm_clear(lsm_t h);

/*
 * lsm_sync -- synchronise the handle's stream and report device-side
 * faults: every wait inside the kernels is bounded, and a wait that ran out
 * (which a correct run never does) is recorded on the device; lsm_sync then
 * returns LSM_EHIP once and clears the record.  LSM_EHIP also for a failed
 * synchronisation.
 */
LSM_API lsm_status_t lsm_sync(lsm_t h);

/*
 * lsm_range_async -- lsm_range without any host synchronisation: always
 * enqueues count, scan and emission.  d_offsets[nq + 1] receives the
 * exclusive scan of the result sizes as in lsm_range; query q writes its
 * pairs only when d_offsets[q + 1] <= cap (all of them, or none), so the
 * caller finds the queries that did not fit by comparing the offsets with
 * cap once the stream has passed the call.  LSM_EINVAL, LSM_ENOMEM,
 * LSM_EHIP.
 */
LSM_API lsm_status_t lsm_range_async(lsm_t h, const uint32_t* d_lo, const uint32_t* d_hi,
                                     uint32_t nq, uint64_t* d_offsets, uint32_t* d_keys,
                                     uint32_t* d_vals, uint64_t cap);

/*
 * lsm_range_async_noalloc -- lsm_range_async for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same outputs, bit for bit,
 * with the per-query counts and the scan's look-back words kept in a fixed
 * array inside the library's code object instead of handle scratch.  The
 * call makes no hipMalloc, hipFree or other allocating call and records no
 * kernel timing.
 *   nq : at most LSM_NOALLOC_MAX_QUERIES; larger batches return
 *        LSM_ECAPACITY with nothing enqueued.
 * The fixed array (4 MiB) exists once per GPU, for the life of the process,
 * and is shared by every handle on that GPU: calls on one GPU whose work
 * overlaps on the device (different streams, not ordered by events) race on
 * it and give undefined output.  Each call clears what it needs, so calls
 * ordered one after another (one stream, or joined by events) are exact.
 * Elements staged by lsm_submit and the pending insertion are completed
 * first, as for every query; when that insertion would need a level or
 * merge buffer the handle has not allocated yet, the call returns
 * LSM_ENOMEM and changes nothing (any query call that may allocate, e.g.
 * lsm_flush, settles it).  Asynchronous.  LSM_EINVAL, LSM_ECAPACITY,
 * LSM_ENOMEM, LSM_EHIP (also when the array's address could not be looked
 * up at lsm_create).
 */
#define LSM_NOALLOC_MAX_QUERIES (1u << 20)
LSM_API lsm_status_t lsm_range_async_noalloc(lsm_t h, const uint32_t* d_lo,
                                             const uint32_t* d_hi, uint32_t nq,
                                             uint64_t* d_offsets, uint32_t* d_keys,
                                             uint32_t* d_vals, uint64_t cap);

/* lsm_destroy -- synchronise the stream and free every allocation. */
LSM_API lsm_status_t lsm_destroy(lsm_t h);

/* ---------------------------------------------------------------------
 * Introspection (tests and measurement; not part of the dictionary).
 * ------------------------------------------------------------------- */

/* Human-readable name of a status code (static string). */
LSM_API const char* lsm_strerror(lsm_status_t s);

/* Number of resident batches r (sec. III-B); 0 for a NULL handle. */
LSM_API uint64_t lsm_num_batches(lsm_t h);

/*
 * Allocation-failure injection, for tests of the strong guarantee: the next
 * n device allocations of the handle succeed and every later one fails as if
 * the device were out of memory (the call then returns LSM_ENOMEM and leaves
 * the dictionary as it was).  A negative n turns the injection off.
 */
LSM_API lsm_status_t lsm_fail_alloc_after(lsm_t h, int64_t n);

/* The batch size b; 0 for a NULL handle. */
LSM_API uint32_t lsm_batch_size(lsm_t h);

/*
 * Device pointers to level i's key variables and values and its length
 * (b * 2^i when occupied, 0 when empty).  Valid until the next update
 * call.  Synchronise the stream before reading them.
 */
LSM_API lsm_status_t lsm_level_view(lsm_t h, uint32_t i, const uint32_t** d_kv,
                            const uint32_t** d_vals, uint64_t* len);

/*
 * Copy level i (occupied) into caller buffers d_kv_out / d_vals_out of
 * b * 2^i elements each, enqueued on the handle's stream.  *len receives
 * the length (0 and nothing copied when level i is empty).
 */
LSM_API lsm_status_t lsm_level_copy(lsm_t h, uint32_t i, uint32_t* d_kv_out,
                                    uint32_t* d_vals_out, uint64_t* len);

typedef struct {
  uint64_t num_batches;        /* r                                        */
  uint64_t resident_elems;     /* r * b                                    */
  uint64_t merged_elems_last;  /* merge output elements of the pairwise
                                  cascade, last update call ((2^(j+1) - 2) b
                                  for an insert into level j; the same
                                  figure when the cascade is fused)         */
  uint64_t merged_elems_total; /* the same, summed since creation           */
  uint64_t sorted_elems_total; /* batch elements sorted since creation     */
  uint64_t device_bytes;       /* device memory held by the handle         */
  uint64_t sorts_top_digit;    /* batch sorts by top-digit scatter + LDS    */
  uint64_t sorts_digit_passes; /* batch sorts by one pass per 8-bit digit   */
} lsm_stats_t;

LSM_API lsm_status_t lsm_get_stats(lsm_t h, lsm_stats_t* out);

/*
 * Device-time profile, gathered while profiling is on (lsm_profile_enable):
 * every kernel is launched between a start and a stop HIP event on the
 * handle's stream (hipExtLaunchKernelGGL), so kernel_ms sums the kernels'
 * own execution times.  lsm_profile_read synchronises the stream, resolves
 * the events and returns the sums since the last reset.
 *
 * Kernel index k: 0 batch-sort histogram (digit-pass path), 1 batch-sort
 * digit pass, 2 level merge, 3 lookup, 4 count, 5 range offset scan, 6 range
 * emission, 7 successor / predecessor, 8 cleanup mark-and-compact, 9 not
 * used (no kernel of this library is counted there), 10 / 11 the top-digit
 * sort's tile scatter and per-bucket sort, 12 the pipelined top-digit sort
 * step (the bucket sort of one batch and the tile scatter of the next in one
 * launch).
 * kernel_bytes[k] is the algorithmic traffic of those launches: 4 B per
 * batch element for a histogram (keys read), 16 B per element for a digit
 * pass, the top-digit scatter and the per-bucket sort (key and value read
 * and written; a per-bucket sort with a fused cascade adds 16 B per element
 * of the levels it takes over), the sum of both for a pipelined step, 16 B
 * per merge output element, 12 B per scanned count; for
 * cleanup 4 B per merged element to count, 8 B per merged element read plus
 * 8 B per valid element written to scatter, 8 B per placebo; 0 for the
 * search kernels, which are latency-bound.
 */
#define LSM_PROF_KERNELS 13
#define LSM_PROF_SIZES 40
typedef struct {
  uint64_t update_calls;                   /* update calls (n > 0)          */
  uint64_t query_calls[3];                 /* lookup, count, range calls    */
  uint64_t query_items[3];                 /* queries answered by each      */
  uint64_t launches[LSM_PROF_KERNELS];     /* launches per kernel           */
  uint64_t elems[LSM_PROF_KERNELS];        /* elements / queries processed  */
  double kernel_ms[LSM_PROF_KERNELS];      /* summed kernel time            */
  double kernel_bytes[LSM_PROF_KERNELS];   /* algorithmic bytes             */
  double update_ms;      /* per update call: first kernel start to last end  */
  double update_p50_ms;
  double update_p99_ms;
  double update_max_ms;
  double query_ms[3];    /* lookup, count, range: first start to last end    */
  /* Level merges (kernel 2) by output size: entry k sums the launches whose
     output holds 2^(k-1) + 1 .. 2^k elements (the cascade's merge into level
     i + 1 of a handle with b = 2^m lands in entry i + 1 + m). */
  uint64_t merge_launches_by_size[LSM_PROF_SIZES];
  double merge_ms_by_size[LSM_PROF_SIZES];
  double merge_bytes_by_size[LSM_PROF_SIZES];
} lsm_profile_t;

LSM_API lsm_status_t lsm_profile_enable(lsm_t h, int on);

/* sizeof(lsm_stats_t) and sizeof(lsm_profile_t), so that a binding can check
 * its copies of the two structures before passing them in. */
LSM_API void lsm_struct_sizes(size_t* stats_size, size_t* profile_size);
LSM_API lsm_status_t lsm_profile_read(lsm_t h, lsm_profile_t* out, int reset);

#ifdef __cplusplus
}
#endif

#endif /* LSM_H_ */
