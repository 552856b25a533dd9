/*
 * pbit.h -- C ABI of the MI355X (gfx950) Pbit list sort.
 *
 * Operation (Planeta, "Pbit and other list sorting algorithms", arXiv
 * cs/0511020, Sec. 3 and Sec. 5): a singly-linked list is re-linked so that
 * it visits its nodes in ascending key order; nodes with equal keys keep the
 * order they had in the input list (stable).  The key is split into M/K
 * patterns of K bits (Sec. 4, digit (key >> s) & (2^K - 1)); the paper splits
 * most-significant pattern first and concatenates the final groups (Sec. 5,
 * merge of Sec. 5.1).  The GPU path produces the same permutation by ranking
 * the list and running stable K-bit passes least-significant first; both are
 * the unique stable sort by the full M-bit key.
 *
 * Data layout (structure of arrays, all DEVICE memory owned by the caller):
 *   next[i]  index of the node after node i, or PBIT_NIL after the last node
 *            (uint32, n entries); the node structure of Sec. 2 split into
 *            arrays.
 *   keys[i]  key of node i, an unsigned M-bit integer stored as uint8_t,
 *            uint16_t, uint32_t or uint64_t for M = 8, 16, 32, 64.
 *   head     index of the first node (Sec. 1, the root), PBIT_NIL if empty.
 * Nodes never move: a payload attached to a node travels with its index.
 *
 * Flags (Sec. 6, Sec. 7-8 and Sec. 14): PBIT_DESCENDING gives the largest
 * key first, PBIT_SIGNED reads keys as two's-complement integers, PBIT_FLOAT
 * reads them as IEEE-754 sign-magnitude numbers of width M (binary16 or
 * bfloat16, binary32, binary64; any 8-bit sign-magnitude format too).
 * Floating-point order is numeric, with -0 before +0 and NaNs outside the
 * infinities on the side of their sign bit (the total order of IEEE-754
 * 2008, Sec. 5.10).  PBIT_SIGNED and PBIT_FLOAT together are PBIT_EINVAL.
 * Equal keys (equal bit patterns) keep list order in every mode.
 *
 * PBIT_SHARED changes no result, only how the digit passes hand out their
 * tiles: by default neighbouring tiles go to one XCD in chunks (their writes
 * merge in that XCD's L2), which assumes the sort has the device to itself;
 * with PBIT_SHARED tiles are claimed in the order blocks start, which stays
 * fast when other kernels (other sorts on other streams) hold parts of the
 * device, at about 10 % more digit-pass time when they do not.
 *
 * Errors are negative return values:
 *   PBIT_EINVAL     bad argument found on the host (no device work queued):
 *                   M not in {8,16,32,64}, K not in {0,1,2,4,8} or not
 *                   dividing M (K = 0: the tuning table picks, see
 *                   pbit_tune_set), n >= 2^32 - 1, head >= n, null pointer,
 *                   an unknown flag bit or PBIT_SIGNED with PBIT_FLOAT,
 *                   workspace too small (see PBIT_ENOMEM);
 *   PBIT_EMALFORMED found on the device: an index >= n, a cycle, or a list
 *                   whose length from head is not n; next[] is left as it
 *                   was (the relink never runs);
 *   PBIT_ENOMEM     workspace smaller than pbit_workspace_bytes();
 *   PBIT_EHIP       a HIP runtime call failed.
 */
#ifndef PBIT_H
#define PBIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PBIT_NIL 0xFFFFFFFFu
/* Largest list: node indices are uint32 with 0xFFFFFFFF as NIL (Sec. 3
 * assumes 32-bit pointers). */
#define PBIT_MAX_NODES 0xFFFFFFFEu

enum {
    PBIT_OK = 0,
    PBIT_EINVAL = -1,
    PBIT_EMALFORMED = -2,
    PBIT_ENOMEM = -3,
    PBIT_EHIP = -4
};

enum {
    PBIT_ASCENDING = 0,
    PBIT_DESCENDING = 1, /* Sec. 6: largest key first                 */
    PBIT_SIGNED = 2,     /* Sec. 7-8: two's-complement keys           */
    PBIT_FLOAT = 4,      /* Sec. 14: IEEE-754 sign-magnitude keys     */
    PBIT_SHARED = 8      /* other kernels may run on the device at the same time */
};

/*
 * Bytes of device workspace needed to sort a list of n nodes with M-bit keys
 * and K-bit patterns (K = 0: the library picks).  Returns 0 for arguments
 * pbit_sort_list_async would reject.  The workspace is O(n): for 32-bit
 * keys about 94 bytes per node up to 2^26 nodes, about 62 up to 2^31 and
 * about 46 beyond (the per-chain slots of the ranking shrink); about 174 for
 * 64-bit keys up to 2^26 nodes.
 */
size_t pbit_workspace_bytes(uint64_t n, uint32_t M, uint32_t K);

/*
 * Sort one list, asynchronously on `stream` (a hipStream_t; NULL = default
 * stream).  Reads next_in[0..n) and keys[0..n); writes the relinked list to
 * next_out[0..n), which may be the same array as next_in (in-place sort).
 * d_result is device memory of two uint32 words that receive
 * {new head, status}; status is PBIT_OK or PBIT_EMALFORMED (as uint32).  On
 * PBIT_EMALFORMED next_out is not written.  ws is device memory of ws_bytes
 * >= pbit_workspace_bytes(n, M, K), used only until the queued work ends.
 * Nothing is allocated; the call may be captured in a HIP graph.  Returns
 * PBIT_OK once the work is queued, or a host-side error (nothing queued).
 */
int pbit_sort_list_async(uint32_t head, const uint32_t *next_in, uint32_t *next_out,
                         const void *keys, uint64_t n, uint32_t M, uint32_t K,
                         uint32_t flags, uint32_t *d_result, void *ws, size_t ws_bytes,
                         void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sort of
 * pbit_sort_list_async with the workspace taken from a fixed array of
 * PBIT_NOALLOC_SCRATCH_BYTES in each device's memory, which the library holds
 * from its first such call on that device until the process ends.  Arguments,
 * result and errors are those of pbit_sort_list_async without ws/ws_bytes;
 * lists whose pbit_workspace_bytes(n, M, K) exceeds the array (about 700 000
 * nodes with 32-bit keys, 380 000 with 64-bit keys) are refused with
 * PBIT_ENOMEM and nothing queued.  The array belongs to the device current at
 * the call, which must be the stream's device.  Nothing is allocated, freed
 * or cleared with a memset: the sort's first kernel zeroes what must start at
 * zero.  All calls on one device share its array: calls whose work may
 * overlap on the device (other streams, or a graph replayed while another
 * runs) race and must be serialised by the caller.
 */
#define PBIT_NOALLOC_SCRATCH_BYTES (64u << 20)
int pbit_sort_list_noalloc(uint32_t head, const uint32_t *next_in, uint32_t *next_out,
                           const void *keys, uint64_t n, uint32_t M, uint32_t K,
                           uint32_t flags, uint32_t *d_result, void *stream);

/*
 * Synchronous, in-place convenience form on the default stream: relinks
 * next[] and returns the new head (PBIT_NIL for an empty list) or a negative
 * status.  Uses a workspace the library keeps between calls (one per device,
 * grown on demand).  next and keys are device pointers.
 */
int64_t pbit_sort_list(uint32_t head, uint32_t *next, const void *keys, uint64_t n,
                       uint32_t M, uint32_t K);

/*
 * Measurement form of pbit_sort_list_async (same arguments and result):
 * events[0..n_events) are hipEvent_t handles created by the caller; the
 * library records events[i] on `stream` before the i-th kernel stage it
 * queues and one more after the last, stores the stage id of each interval
 * in stage_ids (may be NULL) and the number of events recorded in
 * *n_recorded.  Stages beyond n_events - 1 are queued but not bracketed.
 * Used by the benchmark to time each kernel on the stream it runs on.
 */
int pbit_sort_list_profiled(uint32_t head, const uint32_t *next_in, uint32_t *next_out,
                            const void *keys, uint64_t n, uint32_t M, uint32_t K,
                            uint32_t flags, uint32_t *d_result, void *ws, size_t ws_bytes,
                            void *stream, void **events, int32_t *stage_ids, int n_events,
                            int *n_recorded);

/* Name of a stage id reported by pbit_sort_list_profiled ("pack", "walk0",
 * "walk_up", "base", "down", "unchain", "schedule", "digit_pass", "relink",
 * "end"). */
const char *pbit_stage_name(int stage);

/*
 * Many independent lists sorted in one launch sequence (the batched form).
 * The lists share next_in/next_out/keys: list l owns the node slab
 * [d_offsets[l], d_offsets[l+1]) and its next[] entries are global node
 * indices inside that slab (Sec. 3 applied to every list on its own).
 *   d_heads     uint32[num_lists]   first node of each list, PBIT_NIL for an
 *                                   empty slab (device memory)
 *   d_offsets   uint64[num_lists+1] slab bounds, d_offsets[0] = 0,
 *                                   non-decreasing, d_offsets[num_lists] =
 *                                   total_nodes (device memory)
 *   next_in/next_out/keys           as for pbit_sort_list_async, over
 *                                   total_nodes < 2^32 - 1 nodes
 *   d_new_heads uint32[num_lists]   receives each list's new head
 *   d_status    int32               receives PBIT_OK, PBIT_EMALFORMED (some
 *                                   list is not a single NIL-terminated list
 *                                   inside its slab) or PBIT_EINVAL (bad slab
 *                                   bounds or head); on error next_out and
 *                                   d_new_heads are not written
 * Each list comes out exactly as pbit_sort_list_async would sort it alone.
 * ws holds at least pbit_lists_workspace_bytes(total_nodes, num_lists, M, K)
 * bytes.  Nothing is allocated; the call may be captured in a HIP graph.
 * Returns PBIT_OK once queued, or a host-side error (nothing queued).
 */
size_t pbit_lists_workspace_bytes(uint64_t total_nodes, uint32_t num_lists, uint32_t M,
                                  uint32_t K);

int pbit_sort_lists(const uint32_t *d_heads, const uint64_t *d_offsets, uint32_t num_lists,
                    uint64_t total_nodes, const uint32_t *next_in, uint32_t *next_out,
                    const void *keys, uint32_t M, uint32_t K, uint32_t flags,
                    uint32_t *d_new_heads, int32_t *d_status, void *ws, size_t ws_bytes,
                    void *stream);

/*
 * Gather form of pbit_sort_lists for lists that live in separate arrays (a
 * request server batching independent requests without copying them).  List
 * l has len_l = d_offsets[l+1] - d_offsets[l] nodes; its arrays are given by
 * device pointers stored in device memory:
 *   d_next_in_ptrs[l]   uint32[len_l] next[] in LIST-LOCAL indices
 *                       (0..len_l-1, PBIT_NIL at the end)
 *   d_key_ptrs[l]       keys of M bits, len_l entries
 *   d_next_out_ptrs[l]  uint32[len_l] receives the relinked next[] (local
 *                       indices; may equal d_next_in_ptrs[l])
 * d_heads[l] and d_new_heads[l] are list-local too.  d_offsets only sets the
 * lists' places in the workspace.  Results, errors and workspace size are
 * those of pbit_sort_lists with the same offsets.
 */
int pbit_sort_lists_gather(const uint32_t *d_heads, const uint64_t *d_offsets,
                           uint32_t num_lists, uint64_t total_nodes,
                           const uint64_t *d_next_in_ptrs, const uint64_t *d_next_out_ptrs,
                           const uint64_t *d_key_ptrs, uint32_t M, uint32_t K, uint32_t flags,
                           uint32_t *d_new_heads, int32_t *d_status, void *ws, size_t ws_bytes,
                           void *stream);

/* Measurement form of pbit_sort_lists (see pbit_sort_list_profiled). */
int pbit_sort_lists_profiled(const uint32_t *d_heads, const uint64_t *d_offsets,
                             uint32_t num_lists, uint64_t total_nodes, const uint32_t *next_in,
                             uint32_t *next_out, const void *keys, uint32_t M, uint32_t K,
                             uint32_t flags, uint32_t *d_new_heads, int32_t *d_status, void *ws,
                             size_t ws_bytes, void *stream, void **events, int32_t *stage_ids,
                             int n_events, int *n_recorded);

/*
 * Nodes stored as records (the node structure of Sec. 2: the link and the
 * data side by side) instead of separate arrays.  Node i is the record of
 * `stride` bytes at nodes + i * stride (64-bit offsets); its next index is the
 * uint32 at byte next_off of the record and its key the M-bit value at byte
 * key_off.  The two fields must lie inside the record, must not overlap, and
 * must be naturally aligned in every record (stride a multiple of 4 and of the
 * key size, stride < 2^32).  The sort rewrites only the next field of each
 * record, in place; every other byte is left as it was, so the data travels
 * with its node.  Head, keys, flags, d_result, workspace (pbit_workspace_bytes
 * with the same n, M, K), errors and asynchrony are those of
 * pbit_sort_list_async.
 */
int pbit_sort_list_aos_async(uint32_t head, void *nodes, uint64_t stride, uint32_t next_off,
                             uint32_t key_off, uint64_t n, uint32_t M, uint32_t K,
                             uint32_t flags, uint32_t *d_result, void *ws, size_t ws_bytes,
                             void *stream);

/*
 * Doubly-linked lists (Sec. 13).  The sort relinks only next[]; this call then
 * rebuilds the backward links: prev[next[i]] = i for every node i with a
 * successor and prev[h] = PBIT_NIL for every head h in d_heads.  The paper
 * walks each list from its head; since a node's backward link depends only on
 * the forward link into it, the device does it as one scatter over all n
 * nodes, and one call serves a single list or a whole batch.
 *   d_heads    device uint32[num_lists] heads (PBIT_NIL entries are skipped):
 *              the d_result word of pbit_sort_list_async (num_lists = 1) or
 *              the d_new_heads of pbit_sort_lists, used straight after them on
 *              the same stream;
 *   next, prev device uint32[n], distinct arrays; every node must be on one
 *              of the lists (prev of a node on none is not written);
 *   d_status   optional (NULL) device int32: when non-zero on entry (a sort
 *              that found a malformed list) nothing is written; an index >= n
 *              in next[] or d_heads is skipped and sets PBIT_EMALFORMED.
 *              For a single list pass d_result + 1.
 * Asynchronous on `stream`; returns PBIT_EINVAL (n >= 2^32 - 1, null or
 * misaligned pointer, next == prev) with nothing queued, else PBIT_OK or
 * PBIT_EHIP.  Gather-form lists (local indices) are repaired one list at a
 * time with that list's arrays and n = its length.
 */
int pbit_repair_prev_async(const uint32_t *d_heads, uint32_t num_lists, const uint32_t *next,
                           uint32_t *prev, uint64_t n, int32_t *d_status, void *stream);

/*
 * Diagnostic: how long a digit pass's tile waits on a predecessor tile that
 * has not yet published its digit counts (decoupled look-back) before it
 * counts that predecessor's digits in the pass input itself.  `sleeps` is the
 * number of short sleeps per predecessor (default 4096); 0 makes every such
 * tile take the counting path at once.  The result is the same either way;
 * the setting exists so that tests can run the counting path on purpose.  It
 * is process-wide, applies to sorts queued after the call, and returns the
 * previous value.
 */
uint32_t pbit_set_lookback_spin_limit(uint32_t sleeps);

/*
 * Tuning (Sec. 10 weighs the pattern length K against the work per pass;
 * Sec. 9 weighs methods by list length).  When K = 0 is passed, the library
 * picks K, and every sort picks its short-list cutoff, from a table of
 * measured choices: an entry applies to sorts of its kind (0: one list, 1:
 * many lists) and key width M whose node count (for many lists: the total)
 * is at most n_max; the entry with the smallest such n_max wins, else K = 8
 * (4 for M = 8) and cutoff 2048.  Lists of at most `cutoff` nodes in a
 * many-list sort, and a single list of at most `cutoff` nodes (whatever K
 * the caller passes), are each sorted by one workgroup in on-chip memory in
 * one launch; cutoff is 1024, 2048 or 4096.  The result does not depend on
 * the path.  The table is built in (from device measurements) and
 * process-wide.  Records (pbit_sort_list_aos_async) always take the
 * device-wide path.
 *   pbit_tune_set     adds or replaces the entry (kind, M, n_max); returns
 *                     PBIT_OK, PBIT_EINVAL (kind > 1, K not in {1,2,4,8} or
 *                     not dividing M, bad cutoff) or PBIT_ENOMEM (table full)
 *   pbit_tune_clear   empties the table (the defaults above apply)
 *   pbit_tune_reset   restores the built-in table
 *   pbit_tune_lookup  the K and cutoff a sort of that kind, M and size gets
 * Workspace sizes depend on K only, never on the cutoff; a change of the
 * table between pbit_lists_workspace_bytes(.., K = 0) and the sort may change
 * K and so make the workspace too small (PBIT_ENOMEM).
 */
int pbit_tune_set(uint32_t kind, uint32_t M, uint64_t n_max, uint32_t K, uint32_t cutoff);
void pbit_tune_clear(void);
void pbit_tune_reset(void);
int pbit_tune_lookup(uint32_t kind, uint32_t M, uint64_t n, uint32_t *K, uint32_t *cutoff);

/* Human-readable text for a status code. */
const char *pbit_status_string(int code);

/* Library version and build information (static string). */
const char *pbit_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PBIT_H */
