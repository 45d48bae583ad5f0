/*
 * bt.h -- C ABI of libbt: block-tree construction and queries on one MI355X
 * (gfx950) GPU.
 *
 * The method is the per-level construction of Belazzougui et al.'s block tree
 * as described in "Practical Parallel Block Tree Construction: First Results"
 * (Clausecker, Kurpicz, Palanga): Section 4 defines the tree, Section 4.1 its
 * two phases (mark the leftmost occurrence of every pair of consecutive blocks;
 * point every unmarked block at the leftmost occurrence of its content),
 * Section 2 the Karp-Rabin fingerprints used to find candidate occurrences, and
 * Section 1 the access/rank/select queries.  Every fingerprint hit that decides
 * the output is confirmed by comparing bytes, so the tree is exact.
 *
 * Conventions for every entry point
 *   - Return value: BT_OK (0) or a negative BT_E_* status; no exceptions cross
 *     this boundary.  bt_ctx_last_error() gives a message for the last failure.
 *   - Device pointers ("d_" prefix) must point into memory of the context's
 *     device; host pointers ("h_" prefix, or none) are ordinary host memory.
 *   - Work is enqueued on the context's stream.  Builds and queries return after
 *     their device work has completed (the level loop reads per-level counts).
 *     Inputs must stay valid and unmodified until the call returns.
 *   - Positions are 0-based byte offsets; all sizes are in bytes or elements.
 *   - Text bytes are raw uint8 values (the paper's T in [1, sigma]^n, shifted to
 *     0-based symbols).
 *   - A context is used by one host thread at a time.  Finished trees are
 *     read-only; any number of query calls may read them.
 */
#ifndef BT_H
#define BT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define BT_API __attribute__((visibility("default")))
#else
#define BT_API
#endif

/* ---- status codes ---- */
#define BT_OK 0
#define BT_E_INVAL (-1)    /* an argument is out of range (see each call)     */
#define BT_E_NOMEM (-2)    /* a device or host allocation failed               */
#define BT_E_DEVICE (-3)   /* a HIP runtime call failed                        */
#define BT_E_INTERNAL (-4) /* a device-side consistency check failed           */

/* ---- debug flags (bt_params.debug_flags) ---- */
/* Truncate every fingerprint to 12 bits.  Forces fingerprint collisions so that
 * the byte-verification and retry paths run; the output must not change. */
#define BT_DBG_WEAK_HASH 1u
/* Scan with 61-bit fingerprints and without candidate queues, the path that is
 * otherwise taken only past the queues' packing limits (more than 2^24 texts
 * in a batch, or positions beyond 2^40); the output must not change. */
#define BT_DBG_NO_QUEUE 2u
/* Scan every phase with the 32-bit hash pre-filter, also where the byte scan
 * (a filter on each window's first eight bytes, used for phases with few keys)
 * would be taken; the output must not change. */
#define BT_DBG_NO_BYTE_SCAN 4u
/* Find each phase's leftmost occurrences with the sort-based algorithm of
 * Section 5.1 in place of the hash-table scan: every scanned window's and every
 * key's fingerprint sorted together, the first position of each fingerprint
 * broadcast by a scan.  For comparison with hashing; the output must not
 * change.  Needs fewer than 2^31 windows per phase (else BT_E_INVAL) and about
 * 40 bytes of device memory per window. */
#define BT_DBG_SORT_PHASES 8u
/* Batches: scan with one key filter shared by all texts of a phase (the
 * single-text path) instead of a filter per text; the output must not
 * change. */
#define BT_DBG_SHARED_FILTERS 16u

/* ---- build flags (bt_params.flags) ---- */
/* Also build the counters that bt_rank and bt_select need: per block and per
 * symbol, the occurrences before the block; per pointer, the occurrences
 * between its target block's start and its source.  Texts must be shorter than
 * 2^32 bytes.  bt_build always sets it. */
#define BT_WITH_RANK_SELECT 1u
/* Run the optional pruning phase (Section 4.1, after the two phases): marked
 * blocks that no pointer targets become pointers to their leftmost occurrence
 * on the level, deepest internal level first and right to left within a level,
 * when none of their children is marked and that occurrence ends at or before
 * the block and lies in one block or two consecutive ones; their children
 * leave the level below.  The result is the same tree shape with fewer marked
 * blocks (the worked example of Figure 1 is drawn pruned).  The build then
 * scans every block's leftmost occurrence on every level, not only those of
 * unmarked blocks. */
#define BT_PRUNE 2u
/* Memory-lean fingerprints: keep the prefix fingerprints mod 2^61-1 sampled,
 * one value per 16 text bytes (0.5 bytes per text byte instead of 8), and form
 * any other one from its sample and at most 15 text bytes where it is needed
 * (key fingerprints, the scan's candidates, collision retries).  The 32-bit
 * pre-filter hashes stay dense (4 bytes per text byte).  The tree does not
 * change.  Taken when the scan queues its candidates: texts of a batch below
 * 2^24, positions below 2^40, and not BT_DBG_NO_QUEUE; otherwise ignored. */
#define BT_LEAN 4u

typedef struct bt_ctx bt_ctx;   /* device, stream, scratch pool, statistics */
typedef struct bt_tree bt_tree; /* a finished tree, resident in device memory */

/*
 * Build parameters.
 *   tau            inner arity (Section 4: every marked block has tau
 *                  children); >= 2.
 *   leaf_len       block length of the last level, whose blocks are stored
 *                  explicitly (Section 4, stop at |B| in Theta(log_sigma n)); >= 1.
 *   root_block_len 0 to plan by s_hint; otherwise the level-1 block length
 *                  b1, which must equal leaf_len * tau^k for some k >= 0.
 *   s_hint         target root arity s (Section 4, s = z is the space-optimal
 *                  choice): b1 = leaf_len * tau^k with the largest k >= 0 such
 *                  that b1 <= n / s_hint (k = 0 when n / s_hint < leaf_len).
 *                  0 is read as 1.  Then s = ceil(n / b1).
 *   hash_seed      seeds the Karp-Rabin base x in [2^8, 2^61-1); the tree does
 *                  not depend on it.
 *   debug_flags    BT_DBG_* bits.
 *   flags          BT_WITH_RANK_SELECT, BT_PRUNE and BT_LEAN bits, or 0.
 * Block lengths are b_l = b1 / tau^(l-1); the tree has h = k + 1 levels and
 * level h holds the leaves.  Every block has length b_l except the one that
 * ends the text, which may be shorter.
 */
typedef struct {
  uint32_t tau;
  uint32_t leaf_len;
  uint64_t root_block_len;
  uint64_t s_hint;
  uint64_t hash_seed;
  uint32_t debug_flags;
  uint32_t flags;
} bt_params;

/* ---- context ---- */

/* Device memory supplier of a context (the benchmark spec's boundary: the caller's
 * allocator, e.g. PyTorch's caching allocator, provides every device byte the
 * library uses).  alloc returns `bytes` bytes of device memory of the
 * context's device usable on `stream` (the context's stream), or NULL on
 * failure; free returns a block alloc gave.  Both are called from the thread
 * that calls into the library, never concurrently for one context.  The
 * functions and `user` must stay valid until the context and every tree built
 * on it have been released. */
typedef struct {
  void* (*alloc)(void* user, size_t bytes, void* stream);
  void (*free)(void* user, void* ptr, void* stream);
  void* user;
} bt_allocator;

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  The context owns a pool of
 * device memory that grows on demand: blocks come from `allocator` (or from
 * hipMalloc when it is NULL; bt_ctx_create passes NULL), freed blocks are kept
 * for reuse by size, and bt_ctx_trim and bt_ctx_destroy give the cached ones
 * back (trees keep theirs until bt_tree_free).  When the allocator fails, the
 * pool returns its cached blocks and asks once more; a second failure ends the
 * call with BT_E_NOMEM, every block of that call back in the pool.  Errors:
 * BT_E_INVAL (bad device, out == NULL, an allocator without both functions),
 * BT_E_DEVICE, BT_E_NOMEM. */
BT_API int bt_ctx_create(int device, void* hip_stream, bt_ctx** out);
BT_API int bt_ctx_create_ex(int device, void* hip_stream, const bt_allocator* allocator,
                            bt_ctx** out);
BT_API void bt_ctx_destroy(bt_ctx* ctx);
/* Message describing the last failure on this context (never NULL). */
BT_API const char* bt_ctx_last_error(const bt_ctx* ctx);
/* Release pooled scratch memory that is not in use. */
BT_API int bt_ctx_trim(bt_ctx* ctx);

/* Launch and sizing choices of a context's builds.  None of them changes a
 * tree; they trade memory for speed, and their best values depend on the GPU
 * and the shape of the work (paper_2512_23314_amd/autotune.py measures them
 * and keeps the winners per GPU architecture and shape class).
 *   table_load_log2       the key table has at least 2^this slots per key
 *                         (1..3; default 1: load at most 1/2)
 *   text_filter_bits_log2 batches: bits of a text's own key filter per block
 *                         of the level, log2 (4..7; default 5: 32 bits)
 *   span_chunks           batches: windows a workgroup takes at a time, in
 *                         chunks of 1024 (a multiple of 16 up to 1024; 0, the
 *                         default: chosen from the level's size)
 *   filter2_max_log2      single texts: the largest second key filter, log2
 *                         of its bits (16..28; default 24: 2 MiB, L2-sized)
 * Errors: BT_E_INVAL (a value outside its range; the tuning is unchanged). */
typedef struct {
  uint32_t table_load_log2;
  uint32_t text_filter_bits_log2;
  uint32_t span_chunks;
  uint32_t filter2_max_log2;
} bt_tuning;
BT_API int bt_ctx_set_tuning(bt_ctx* ctx, const bt_tuning* tuning);
BT_API int bt_ctx_get_tuning(const bt_ctx* ctx, bt_tuning* tuning);

/* Per-kernel timing, measured with HIP events on the context's stream around
 * each launch of the named kernel while enabled.  `bytes` accumulates the
 * kernel's algorithmic traffic (the bytes the method must move; defined with
 * each kernel in the design notes) and `units` its work units (windows for the
 * probe scan, text bytes for the prefix scan).  Names: "prefix_fp" (the
 * prefix scan: fingerprints and, in builds, the 32-bit hashes), "probe_scan",
 * "byte_scan", "verify", "sort_phase". */
BT_API int bt_ctx_profile(bt_ctx* ctx, int enable);
BT_API int bt_ctx_kernel_stats(const bt_ctx* ctx, const char* name, uint64_t* launches,
                        double* total_ms, double* bytes, double* units);
BT_API int bt_ctx_reset_stats(bt_ctx* ctx);
/* The same timed launches one by one, in launch order, since the last
 * bt_ctx_reset_stats (at most 65536 are kept).  For launch idx < count: the
 * kernel name (NUL-terminated, cut to name_cap - 1 characters), the window
 * length L of a scan launch (0 for other kernels), its work units, HIP-event
 * milliseconds and algorithmic bytes.  For "probe_scan" the algorithmic bytes
 * are those of the prefix values its tiles must read: a tile of 1024
 * consecutive windows reads values [i0, i0 + 1024) and [i0 + L, i0 + L + 1024),
 * 4 bytes each (8 without the 32-bit pre-filter), and the union is counted,
 * i.e. 4 (1 + min(L, 1024) / 1024) bytes per window.  Any output may be NULL.
 * Errors: BT_E_INVAL (idx out of range). */
/* Per-phase device counters of the builds run while profiling, since the last
 * bt_ctx_reset_stats, in order (at most 65536 kept).  Record idx < count, nine
 * words:
 *   rec[0] level step (0-based; a batch's texts share steps by block length),
 *   rec[1] block length b, rec[2] phase (1: pairs of blocks, 2: blocks),
 *   rec[3] blocks of the level (all texts), rec[4] keys inserted into the table
 *   (keys the level above proved to be copies stay out), rec[5] windows
 *   scanned, rec[6] windows that passed the scan's filters and probed the
 *   table, rec[7] keys verified against the text (their leftmost hit is not
 *   their own start), rec[8] collisions: verifications that failed (a
 *   fingerprint collision, or a hit in another text of the batch), each then
 *   resolved by the exact retry walk.
 * Errors: BT_E_INVAL (idx out of range). */
BT_API int bt_ctx_phase_count(const bt_ctx* ctx, uint64_t* count);
BT_API int bt_ctx_phase_record(const bt_ctx* ctx, uint64_t idx, uint64_t* rec);
BT_API int bt_ctx_launch_count(const bt_ctx* ctx, uint64_t* count);
BT_API int bt_ctx_launch_record(const bt_ctx* ctx, uint64_t idx, char* name, uint64_t name_cap,
                                uint64_t* window_len, double* units, double* ms, double* bytes);
/* Device memory of the context's pool, in bytes: handed out and not yet
 * returned (scratch of a build in flight plus the storage of live trees), the
 * most of that since the last bt_ctx_reset_peak, and all that the pool holds
 * (cached blocks included).  Any output may be NULL.  Errors: BT_E_INVAL. */
BT_API int bt_ctx_memory(const bt_ctx* ctx, uint64_t* in_use, uint64_t* peak, uint64_t* held);
BT_API int bt_ctx_reset_peak(bt_ctx* ctx);

/* ---- step (a2) on its own: prefix fingerprints ----
 * Section 2, the Karp-Rabin fingerprint phi, with q = 2^61-1 and r = x:
 *   d_P[0] = 0,  d_P[i+1] = (d_P[i] * x + d_text[i]) mod (2^61 - 1),
 * so that the fingerprint of T[i..i+L) is (P[i+L] - P[i] * x^L) mod q.
 * d_text: n bytes (device).  d_P: n+1 uint64 (device, caller-owned).
 * x must be in [1, 2^61-1).  Errors: BT_E_INVAL. */
BT_API int bt_prefix_fingerprints(bt_ctx* ctx, const uint8_t* d_text, uint64_t n, uint64_t x,
                           uint64_t* d_P);

/* ---- both prefix arrays of a build, in one pass ----
 * The fingerprints of bt_prefix_fingerprints (base x) and the 32-bit
 * pre-filter hashes of the probe scan (a bit filter on these prunes windows
 * before any fingerprint is formed, Section 4.1 step a4):
 *   d_H[0] = 0,  d_H[i+1] = (d_H[i] * x32 + d_text[i]) mod 2^32.
 * sampled = 0: d_P holds n+1 uint64 as in bt_prefix_fingerprints;
 * sampled = 1: d_P[q] = P[16 q] for 16 q <= n (n/16 + 1 uint64), and d_H
 * holds n+1 uint32;
 * sampled = 2: both sampled, d_P as for 1 and d_H[q] = H[16 q] (n/16 + 1
 * uint32), the form a memory-lean build keeps.  All device, caller-owned.
 * x must be in [1, 2^61-1); any x32.  Errors: BT_E_INVAL (also for sampled
 * outside 0..2). */
BT_API int bt_prefix_scan(bt_ctx* ctx, const uint8_t* d_text, uint64_t n, uint64_t x,
                          uint32_t x32, int sampled, uint64_t* d_P, uint32_t* d_H);

/* ---- the same pass without allocating ----
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Arguments,
 * outputs and errors are those of bt_prefix_scan; the caller still provides
 * d_text, d_P and d_H.  The scan's own scratch (its power tables and the
 * look-back status words, which bt_prefix_scan takes from the context's pool)
 * lives in a fixed device array of the library, BT_NOALLOC_SCRATCH_BYTES on
 * each GPU the library runs on, held until the process ends.  That array
 * bounds n: more than BT_NOALLOC_MAX_TEXT bytes -> BT_E_INVAL, before any
 * device work.  The call allocates nothing (no hipMalloc or hipFree, no
 * pooled buffer) and returns after its device work has completed.  Calls on
 * one GPU share its array: calls that overlap on one GPU (from several host
 * threads, or on several streams) race; calls ordered on one stream do not.
 * Errors: BT_E_INVAL, BT_E_DEVICE (also when the array could not be located
 * on this device when the context was created). */
#define BT_NOALLOC_MAX_TEXT (1ull << 33)
/* an upper bound on the array's size (4 MiB of status words plus the tables) */
#define BT_NOALLOC_SCRATCH_BYTES ((4u << 20) + (128u << 10))
BT_API int bt_prefix_scan_noalloc(bt_ctx* ctx, const uint8_t* d_text, uint64_t n, uint64_t x,
                                  uint32_t x32, int sampled, uint64_t* d_P, uint32_t* d_H);

/* ---- builds ----
 * Build the block tree of the n bytes at d_text (device, caller-owned).
 * sigma is an upper bound on the number of distinct byte values (1..256); it
 * sizes the rank/select support and is checked: more distinct values than
 * sigma -> BT_E_INVAL.  n = 0 gives an empty tree with one (leaf) level.
 * On success *out receives a tree owned by the caller (free with
 * bt_tree_free).  Errors: BT_E_INVAL (tau < 2, leaf_len = 0, sigma outside
 * 1..256, a bad root_block_len, out == NULL), BT_E_NOMEM, BT_E_DEVICE,
 * BT_E_INTERNAL. */
BT_API int bt_build(bt_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t sigma, uint32_t tau,
             uint32_t leaf_len, bt_tree** out);
BT_API int bt_build_ex(bt_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t sigma,
                const bt_params* params, bt_tree** out);

/* Build `num` independent trees in one pass: text i is
 * d_concat[h_offsets[i] .. h_offsets[i+1]) (h_offsets: num+1 host values,
 * non-decreasing, h_offsets[0] may be > 0).  All texts share params (each text
 * gets its own b1 from its own length).  Levels of every text with the same
 * block length are processed by the same kernel launches.  Tree i equals
 * bt_build_ex of text i with the same params.  outs: num host slots.
 * Errors: as bt_build_ex; on failure no tree is returned. */
BT_API int bt_build_batch(bt_ctx* ctx, const uint8_t* d_concat, const uint64_t* h_offsets,
                   uint32_t num, uint32_t sigma, const bt_params* params, bt_tree** outs);

/* ---- tree inspection (the stored structure: Section 5.4, one bit vector
 *      of marks per level plus pointers and offsets) ---- */

/* n, the number of levels h (>= 1), and b1. */
BT_API int bt_tree_info(const bt_tree* tree, uint64_t* n, uint32_t* h, uint64_t* b1);
/* Level l in 1..h: block length b, number of blocks c, number of unmarked
 * blocks u (0 on level h).  Errors: BT_E_INVAL for l outside 1..h. */
BT_API int bt_level_info(const bt_tree* tree, uint32_t level, uint64_t* b, uint64_t* c, uint64_t* u);
/* Copy level l (< h) to host buffers (any may be NULL):
 *   marked_words  ceil(c/64) uint64, bit j%64 of word j/64 = block j marked
 *                 (LSB first, pad bits zero)
 *   ptr_block     u uint64: for the k-th unmarked block (in block order), the
 *                 index among this level's blocks of the block holding the
 *                 first byte of the leftmost occurrence of its content
 *   ptr_off       u uint64: offset of that occurrence inside that block
 * Errors: BT_E_INVAL for l outside 1..h-1. */
BT_API int bt_level_copy(const bt_tree* tree, uint32_t level, uint64_t* marked_words,
                  uint64_t* ptr_block, uint64_t* ptr_off);
/* The same copy enqueued on `stream` (a hipStream_t of the tree's device; NULL
 * = the null stream) into host or device destinations, returning without
 * waiting: the destinations hold the level once the stream reaches this point
 * (pinned or device destinations; a pageable host destination makes the copy
 * synchronous).  Errors: BT_E_INVAL, BT_E_DEVICE. */
BT_API int bt_level_copy_async(const bt_tree* tree, uint32_t level, uint64_t* marked_words,
                               uint64_t* ptr_block, uint64_t* ptr_off, void* stream);
/* Number of leaf bytes (the sum of the level-h block lengths) and a copy of
 * them, block by block, into a host buffer. */
BT_API int bt_leaves_size(const bt_tree* tree, uint64_t* bytes);
BT_API int bt_leaves_copy(const bt_tree* tree, uint8_t* dst);

/* Canonical little-endian serialisation, compared byte for byte in tests:
 *   "BTv1", u64 n, u32 tau, u32 leaf_len, u64 b1, u32 h, u32 0,
 *   for each level l < h: u64 b, u64 c, ceil(c/64) u64 mark words, u64 u,
 *                         u64 ptr_block[u], u64 ptr_off[u]
 *   level h: u64 b, u64 c, u64 leaf byte count, the leaf bytes, zero padding
 *            to a multiple of 8.
 * With dst == NULL only *written (the size) is set.  Errors: BT_E_INVAL when
 * cap is too small. */
BT_API int bt_serialize(const bt_tree* tree, uint8_t* dst, uint64_t cap, uint64_t* written);

/* ---- queries (Section 1), batched; all arrays are device memory ----
 *   access(i)    = T[i]                               for i in [0, n)
 *   rank(c, i)   = #{ j < i : T[j] = c }              for i in [0, n]
 *   select(c, k) = position of the k-th occurrence of c, k >= 1
 * (rank is the paper's rank_c(i) with 1-based inclusive positions; select is
 * the paper's select minus one.)  Out-of-range i, k = 0 or k > count(c) give
 * UINT64_MAX; access of an out-of-range i gives 0 and the call returns
 * BT_E_INVAL after answering the rest.  bt_rank and bt_select return
 * BT_E_INVAL when the tree was built without BT_WITH_RANK_SELECT. */
BT_API int bt_access(bt_ctx* ctx, const bt_tree* tree, const uint64_t* d_pos, uint64_t m,
              uint8_t* d_out);
BT_API int bt_rank(bt_ctx* ctx, const bt_tree* tree, const uint8_t* d_c, const uint64_t* d_pos,
            uint64_t m, uint64_t* d_out);
BT_API int bt_select(bt_ctx* ctx, const bt_tree* tree, const uint8_t* d_c, const uint64_t* d_k,
              uint64_t m, uint64_t* d_out);

/* Device bytes held by a tree (for a tree of a batch: the batch's storage
 * divided by the number of trees). */
BT_API int bt_tree_device_bytes(const bt_tree* tree, uint64_t* bytes);
/* Of those, the bytes of the rank/select support (0 without
 * BT_WITH_RANK_SELECT; same division for a batch).  The support keeps, per
 * level and symbol, each block's count relative to its parent block in 8 or 16
 * bits (absolute 32-bit counts on a tree's first level and where relative ones
 * would need 32 bits), pointer counts in 8, 16 or 32 bits, the index of every
 * marked block and the block starts. */
BT_API int bt_tree_rank_bytes(const bt_tree* tree, uint64_t* bytes);
BT_API void bt_tree_free(bt_tree* tree);
/* bt_tree_free of trees[0 .. n) (null entries are skipped): one call for the
 * trees of a batch.  Errors: BT_E_INVAL (trees null with n > 0). */
BT_API int bt_trees_free(bt_tree* const* trees, uint64_t n);
BT_API const char* bt_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* BT_H */
