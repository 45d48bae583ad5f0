// Internal interface between the host orchestration (bt_host.cpp) and the HIP
// kernels (*.hip).  Plain structs of device pointers and sizes; every launch
// wrapper enqueues on the given stream and returns the launch status.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bt {

// ---- prefix fingerprints (step a2) ----
constexpr int kPfThreads = 512;
constexpr int kPfBytes = 64;                            // consecutive bytes per thread
constexpr uint64_t kPfTile = kPfThreads * kPfBytes;     // bytes per tile (32 KiB)

// Tables of the prefix scan for one pair of bases, computed on the host: x mod
// 2^61-1 (the fingerprints) and x32 mod 2^32 (the pre-filter hashes).
struct PfTab {
  uint64_t g61[7][256];          // b x^j mod 2^61 - 1, j = 1..7 (row j - 1), b = 0..255
  uint64_t t61[kPfThreads + 1];  // x^(64 k), k = 0..256
  uint64_t xt61[65];             // x^(tile k), k = 0..64
  uint64_t c61[4];               // x^(16 c), c = 0..3
  uint64_t x1_61, x8_61;         // x, x^8
  uint32_t t32[kPfThreads + 1];
  uint32_t xt32[65];
  uint32_t c32[4];
  uint32_t x1_32, x8_32;
};

// Status words of the prefix scan's look-back for n text bytes: two arrays of
// tiles + 1 words and the tile counter.  The launch wrapper zeroes them.
inline uint64_t prefix_status_words(uint64_t n) {
  return 2 * ((n + kPfTile - 1) / kPfTile + 1) + 1;
}

// P[0] = 0, P[i+1] = P[i] x + T[i] (mod 2^61 - 1) for i < n, stored dense
// (n + 1 words) or, when sampled, as Ps[q] = P[16 q] for 16 q <= n (n / 16 + 1
// words), or with quarter (not sampled) as Ps[q] = P[4 q] for 4 q <= n (n / 4 +
// 1 words); and, when H is not null, H[0] = 0, H[i+1] = H[i] x32 + T[i] (mod
// 2^32), the pre-filter hashes of the probe scan (n + 1 words), from the same
// pass over the text; hsampled (with sampled): H holds H[16 q] for 16 q <= n
// instead (n / 16 + 1 words).  status: prefix_status_words(n) words.
hipError_t launch_prefix(const uint8_t* T, uint64_t n, uint64_t* P, bool sampled, uint32_t* H,
                         const PfTab* tab, uint64_t* status, hipStream_t s, bool hsampled = false,
                         bool quarter = false);

// ---- level data (device arrays; positions are offsets into the text base) ----
struct TextsDev {
  uint32_t T;              // number of texts
  const uint64_t* tstart;  // [T]
  const uint64_t* tend;    // [T]
  const uint64_t* tsalt;   // [T]
};

struct LevelDev {
  uint64_t c;              // blocks
  uint64_t b;              // block length
  const uint64_t* st;      // [c] block starts, increasing
  const uint32_t* text;    // [c] text of each block
  const uint32_t* run;     // [c] run of each block
  uint64_t R;              // runs (maximal sequences of consecutive blocks)
  const uint64_t* rs;      // [R] run start
  const uint64_t* re;      // [R] run end
  const uint32_t* rtext;   // [R]
};

// Keys of one phase.  Keys are indexed by block: block j carries the key of
// the pair (j, j+1) in phase 1 and of its own content in phase 2.
struct KeysDev {
  uint64_t* fp;     // [c]
  uint64_t* len;    // [c]
  uint32_t* slot;   // [c] table slot, kNoKey, kOddKey or kCopyKey
  uint64_t* lm;     // [c] leftmost occurrence (result)
};

// Keys whose length differs from the phase's main length (at most one per
// text: the one ending at the text's end).  Indexed by text.
struct OddDev {
  uint64_t* L;      // [T] 0 = none
  uint64_t* xp;     // [T] x^L
  uint64_t* fp;     // [T]
  uint64_t* best;   // [T] atomicMin target, initialised to the key's position
  uint64_t* pos;    // [T]
  uint64_t* nkeys;  // [T] keys of this text in this phase (main + odd)
  uint64_t* h32;    // [T] the key's 32-bit hash (low half) and x32^L (high half)
};

struct Slot {
  uint64_t fp;
  uint64_t best;  // smallest position with this fingerprint seen so far
};

// Open addressing with linear probing; an empty slot has fp = kEmpty.
struct TableDev {
  Slot* slots;
  uint64_t mask;  // capacity - 1 (capacity a power of two, at least 1024)
};

struct PhaseArgs {
  const uint8_t* T;
  const uint64_t* P;      // prefix fingerprints by text position, or null when sampled:
  const uint64_t* Ps;     // Ps[q] = P[pbase + 2^pshift q]
  uint32_t pshift;        // 4 (memory-lean builds), or 2 (dense 32-bit hashes beside them)
  uint64_t pbase;
  uint64_t pend;          // end of the text bytes (offset), for the lean loads
  TextsDev tx;
  LevelDev lv;
  KeysDev k;
  OddDev odd;
  TableDev tab;
  uint64_t Lmain;   // standard key length (2b in phase 1, b in phase 2)
  uint64_t xLmain;  // x^Lmain
  uint64_t x;
  uint64_t fpmask;  // all ones, or kWeakMask
  const uint8_t* marked;  // phase 2: skip marked blocks
  int phase;        // 1 or 2
  uint32_t* filt;   // bit filter of the main-length keys' fingerprints
  uint32_t filt_bits;  // log2 of its size in bits (12..19); 0 = no filter
  uint32_t filt_two;   // 1: two bits per key, 0: one
  uint32_t all_blocks; // phase 2: keys for every block, not only unmarked ones
  // 32-bit pre-filter hash: when pre32 is set the filter holds bits of the
  // keys' 32-bit window hashes, and the scan computes a window's fingerprint
  // only where its 32-bit hash passes the filter.
  const uint32_t* P32;  // prefix hashes mod 2^32 (same indexing as P), or null when sampled:
  const uint32_t* Hs;   // Hs[q] = H[pbase + 16 q] (memory-lean builds)
  uint32_t x32L;        // x32^Lmain mod 2^32
  uint32_t x32Lm1;      // x32^(Lmain - 1): the weight of the byte that leaves a rolled window
  uint32_t x32inv;      // x32^-1 mod 2^32 (x32 is odd)
  uint32_t x32;         // the 32-bit hash's base
  uint32_t pre32;
  // With pre32: a second, blocked bit filter of the keys' 32-bit hashes in
  // global memory (2^filt2_words 64-bit words, three bits of one word per key;
  // 0 = none), tested by the windows that pass the LDS filter before they are
  // queued.
  uint32_t* filt2;
  uint32_t filt2_words;
  // Facts about each block's parent (kSkip* of its scan entry, plus
  // kLastChild), or null.  A key whose string lies inside a parent region that
  // the level above proved to be a copy is not inserted (kCopyKey).
  const uint8_t* cflag;
  uint32_t exact_all;  // phase 2 over all blocks needs every block's exact leftmost occurrence
  // Byte scan (few keys, all at least 8 bytes long): a bit filter of the keys'
  // first eight bytes (2^bfilt_bits bits, 0 = off), tested on the text itself.
  uint32_t* bfilt;
  uint32_t bfilt_bits;
  // Text-local filters (batches, with pre32): per text t, a blocked filter of
  // its keys' 32-bit hashes, 2^tf_wl[t] 32-bit words at tf_words + tf_off[t],
  // three bits of one word per key (tfilter_word, tfilter_mask).  Null when off.
  uint32_t* tf_words;
  const uint64_t* tf_off;  // [T]
  const uint32_t* tf_wl;   // [T], at least 3
  // For a text whose filter is larger than LDS (tf_wl[t] > F, F =
  // kTextFilterLdsLog2): the same filter folded to 2^F words at tf_fold +
  // tf_fold_off[t] (word k = OR of the 2^(wl - F) words
  // k 2^d .., a superset test: a window failing it fails the full filter).
  uint32_t* tf_fold;
  const uint64_t* tf_fold_off;  // [T] (read only for such texts)
  // Counters of this phase (profiling only, else null): [kPcKeys] keys
  // inserted by k_keys, [kPcCand] windows that passed the scan's filters.
  uint64_t* pc;
};
// Words per phase record: keys inserted, candidates, windows scanned, keys
// verified (hit elsewhere than at their own start), collisions (verification
// failed: the exact retry ran).
constexpr int kPcKeys = 0, kPcCand = 1, kPcWindows = 2, kPcVerified = 3, kPcCollisions = 4;
constexpr int kPcWords = 8;

// Scan entries and segments (level.hip, "scan segments").
constexpr uint8_t kSkipInterior = 1;  // windows ending inside the entry are copies
constexpr uint8_t kSkipCross = 2;     // every window starting in the entry is a copy
constexpr uint8_t kLastChild = 4;     // (per block) the last child of its parent
struct SegDev {
  uint64_t E;             // entries
  const uint64_t* ea;     // [E] entry start
  const uint64_t* ee;     // [E] entry end
  const uint8_t* ef;      // [E] kSkip* flags
  const uint32_t* erun;   // [E] run of the entry
  uint64_t* ws;           // [E] first window start of the segment
  uint64_t* sre;          // [E] run end
  uint32_t* stext;        // [E] text
};

hipError_t launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, uint64_t n, hipStream_t s);
// Up to kFillJobs fills of 32-bit words in one launch (jobs with no words are
// skipped by their blocks).
constexpr int kFillJobs = 8;
struct FillList {
  uint32_t* p[kFillJobs];
  uint64_t words[kFillJobs];
  uint32_t value[kFillJobs];
  int n = 0;
  void add(void* ptr, uint64_t nwords, uint32_t v) {
    p[n] = static_cast<uint32_t*>(ptr);
    words[n] = nwords;
    value[n] = v;
    ++n;
  }
};
hipError_t launch_fill_many(const FillList& f, hipStream_t s);

// Exclusive scan of a[0..n) in place; a[n] receives the total.  tmp must hold
// scan_tmp_words(n) words.
uint64_t scan_tmp_words(uint64_t n);
hipError_t scan_excl_u64(uint64_t* a, uint64_t n, uint64_t* tmp, hipStream_t s);
// Per-text counts of the next level in one launch, for T <= kTextStepMax texts:
// ncount[t] = cs[tfirst[t] + tcount[t]] - cs[tfirst[t]] + enter[t];
// nfirst = exclusive prefix of ncount (T + 1 words);
// tu[t] = uoff[tfirst[t] + tcount[t]] - uoff[tfirst[t]].
constexpr uint32_t kTextStepMax = 2048;
hipError_t launch_text_step(uint32_t T, const uint64_t* cs, const uint64_t* tfirst,
                            const uint64_t* tcount, const uint64_t* enter, const uint64_t* uoff,
                            uint64_t* ncount, uint64_t* nfirst, uint64_t* tu, hipStream_t s);

// The probe scan's tile: a wave takes this many consecutive window numbers at
// a time (lanes step through them 64 apart).
constexpr uint64_t kProbeTile = 1024;

// Phase kernels (steps a3-a7).
hipError_t launch_keys(const PhaseArgs& a, hipStream_t s);
hipError_t launch_entries_from_runs(const LevelDev& lv, uint64_t* ea, uint64_t* ee, uint8_t* ef,
                                    uint32_t* erun, hipStream_t s);
hipError_t launch_pair_facts(const PhaseArgs& a, uint8_t* pf, hipStream_t s);
hipError_t launch_block_facts(const PhaseArgs& a, uint8_t* pf, hipStream_t s);
hipError_t launch_entries_next(const LevelDev& lv, const TextsDev& tx, const uint8_t* marked,
                               const uint8_t* pf, const uint64_t* uoff, const uint64_t* cs,
                               const uint64_t* tfirst, const uint64_t* ntfirst, uint64_t nmarked,
                               const uint32_t* ids, uint32_t E, uint64_t* ea, uint64_t* ee,
                               uint8_t* ef, uint64_t* echild, hipStream_t s);
hipError_t launch_entry_runs(const uint64_t* echild, uint64_t E, const uint32_t* run,
                             uint32_t* erun, hipStream_t s);
// Per-block parent facts from the level's entries: cflag (c bytes, zeroed by
// the caller) gets the entry's kSkip* flags on each child of a flagged entry,
// plus kLastChild on its last child.  b: this level's block length.
hipError_t launch_child_flags(const SegDev& sg, uint64_t b, const uint64_t* echild, uint8_t* cflag,
                              hipStream_t s);
// Per-segment window counts into woff[0..E) (then scanned by the caller).
hipError_t launch_segments(const PhaseArgs& a, const SegDev& sg, uint64_t* woff, hipStream_t s);
// Phase-1 segments merged where one entry's window starts continue the previous
// entry's (see level.hip): head[0..E) then scanned by the caller (total at E),
// then the merged arrays, E of them (E + 1 offsets), padded past the last.
hipError_t launch_seg_heads(const SegDev& sg, const uint64_t* woff, uint64_t* head, hipStream_t s);
hipError_t launch_seg_merge(const SegDev& sg, const uint64_t* woff, const uint64_t* hs, uint64_t* ws,
                            uint64_t* sre, uint32_t* stext, uint64_t* woff2, hipStream_t s);
// Phase-2 segments from this level's pair facts (bit 0 of pf); see level.hip.
hipError_t launch_block_seg_counts(const PhaseArgs& a, const uint8_t* pf, uint64_t* wc,
                                   uint64_t* head, hipStream_t s);
hipError_t launch_block_segments(const PhaseArgs& a, const uint64_t* wcs, const uint64_t* hs,
                                 uint64_t* ws, uint64_t* sre, uint32_t* stext, uint64_t* woff,
                                 hipStream_t s);
// Sort-based phases (sort_phase.hip): windows and keys as (fingerprint,
// position or key block), sorted by fingerprint; none marks entries that match
// nothing (above every fingerprint).
hipError_t launch_sort_emit(const PhaseArgs& a, const uint64_t* woff, uint64_t W, uint64_t none,
                            uint64_t* fpv, uint64_t* posv, hipStream_t s);
// hipCUB's stable radix sort of n pairs by the low end_bit key bits; with tmp
// null it only sets tmp_bytes.
hipError_t sort_pairs_u64(void* tmp, size_t& tmp_bytes, const uint64_t* kin, uint64_t* kout,
                          const uint64_t* vin, uint64_t* vout, uint64_t n, int end_bit,
                          hipStream_t s);
hipError_t launch_sort_heads(const uint64_t* fp, uint64_t n, uint64_t* h, hipStream_t s);
// gx: exclusive scan of the head flags; gfirst: n words
hipError_t launch_sort_groups(const PhaseArgs& a, const uint64_t* fp, const uint64_t* pos,
                              const uint64_t* gx, uint64_t n, uint64_t* gfirst, hipStream_t s);
// The byte scan: every window's first eight text bytes against the keys'
// prefix filter; windows that pass form their fingerprint and probe the table.
hipError_t launch_byte_scan(const PhaseArgs& a, const uint64_t* woff, bool has_odd, bool has_salt,
                            uint64_t max_windows, hipStream_t s);
// The sliding-window probe.  max_windows bounds the grid; mode 0: no filter,
// 1: LDS key filter and per-wave candidate queues, 2: LDS key filter, inline probe.
hipError_t launch_probe_scan(const PhaseArgs& a, const uint64_t* woff, bool has_odd,
                             bool has_salt, uint64_t max_windows, int mode, hipStream_t s);
// The probe scan of a batch with text-local filters (probe_text.hip): resident
// workgroups take spans of span_chunks * kProbeTile windows from *span_ctr
// (zeroed by the caller); a window is tested against its own text's filter,
// from LDS when the span lies in one text (its filter, or the folded filter of
// a text whose filter does not fit, then the full one in global memory).
// Needs pre32, text-local filters, salts, and span_info as launch_span_info
// left it (same window bound and span length).
uint64_t probe_text_spans(uint64_t max_windows, uint64_t span_chunks);
// Each span's first and last segment and its text (or none), three words per
// span into span_info (3 * probe_text_spans(...) words).
hipError_t launch_span_info(const PhaseArgs& a, const uint64_t* woff, uint64_t max_windows,
                            uint64_t span_chunks, uint64_t* span_info, hipStream_t s);
// short_segments: the segments are expected to be short against a tile (the
// scan then walks them from registers; dense hashes only).
hipError_t launch_probe_text(const PhaseArgs& a, const uint64_t* woff, bool has_odd,
                             uint64_t max_windows, uint64_t span_chunks, uint64_t* span_ctr,
                             const uint64_t* span_info, bool short_segments, hipStream_t s);
// Folds the filters of the nbig texts listed in big (see PhaseArgs.tf_fold).
hipError_t launch_fold_filters(const PhaseArgs& a, const uint32_t* big, uint32_t nbig,
                               hipStream_t s);
// log2 of the 32-bit words of the largest text-local filter a span loads into
// LDS: 128 KiB (the scan runs one 1024-thread workgroup per CU, which leaves
// room for the filter and the queues in the CU's 160 KiB).
constexpr uint32_t kTextFilterLdsLog2 = 15;

struct VerifyBufs {
  uint32_t* vlist;  // [c]
  uint64_t* vbest;  // [c]
  uint32_t* vmis;   // [c]
  uint32_t* rlist;  // [c]
  uint64_t* rlb;    // [c]
  uint64_t* counts; // [2]: verify count, retry count
};
hipError_t launch_resolve(const PhaseArgs& a, const VerifyBufs& v, hipStream_t s);
// Profiling: copy the phase's window count and verification counts into pc.
hipError_t launch_phase_record(uint64_t* pc, const uint64_t* windows, const VerifyBufs& v,
                               hipStream_t s);
hipError_t launch_verify(const PhaseArgs& a, const VerifyBufs& v, uint64_t max_len,
                         hipStream_t s);
hipError_t launch_finish(const PhaseArgs& a, const VerifyBufs& v, hipStream_t s);
hipError_t launch_retry(const PhaseArgs& a, const VerifyBufs& v, hipStream_t s);

// Step a5: marks from the phase-1 results (plus the isolated-block rule).
hipError_t launch_mark(const PhaseArgs& a, uint8_t* marked, hipStream_t s);
// marks, pair facts (bit 0), the unmarked indicator and the next level's run
// starts in one pass
hipError_t launch_mark_facts(const PhaseArgs& a, uint8_t* marked, uint8_t* pf, uint64_t* ucnt,
                             uint64_t* nrun, hipStream_t s);
// Unmarked-prefix counts: cnt[j] = !marked[j].
hipError_t launch_unmarked_counts(const uint8_t* marked, uint64_t c, uint64_t* cnt,
                                  hipStream_t s);
// Step a7: pointers.  uoff = exclusive scan of unmarked counts; tfirst = first
// block of each text on this level.  err receives 1 on a broken invariant.
hipError_t launch_pointers(const PhaseArgs& a, const uint8_t* marked, const uint64_t* uoff,
                           const uint64_t* tfirst, uint64_t* ptr_block, uint64_t* ptr_off,
                           uint32_t* err, hipStream_t s);

// Step a8: split.
hipError_t launch_child_counts(const LevelDev& lv, const TextsDev& tx, const uint8_t* marked,
                               uint64_t bn, uint64_t* cnt, hipStream_t s);
// Per-text next-level counts: children (from the scanned child counts) plus
// entering blocks.  tcount/tfirst describe the current level.
hipError_t launch_text_counts(uint32_t T, const uint64_t* cs, const uint64_t* tfirst,
                              const uint64_t* tcount, const uint64_t* enter,
                              uint64_t* ncount, hipStream_t s);
hipError_t launch_write_children(const LevelDev& lv, const TextsDev& tx, const uint8_t* marked,
                                 uint64_t bn, uint32_t tau, const uint64_t* cs,
                                 const uint64_t* tfirst, const uint64_t* ntfirst,
                                 uint64_t* nst, uint32_t* ntext, hipStream_t s);
hipError_t launch_write_entering(const uint32_t* ids, uint32_t E, const TextsDev& tx,
                                 uint64_t bn, const uint64_t* ntfirst, uint64_t* nst,
                                 uint32_t* ntext, hipStream_t s);
// Runs of a level: flags into rflag (c entries, then scanned by the caller).
hipError_t launch_run_flags(const uint64_t* st, const uint32_t* text, uint64_t c, uint64_t b,
                            uint64_t* rflag, hipStream_t s);
// From the scanned flags (exclusive; roff[c] = R): run ids and the run table.
hipError_t launch_run_table(const uint64_t* st, const uint32_t* text, uint64_t c, uint64_t b,
                            const TextsDev& tx, const uint64_t* roff, uint32_t* run,
                            uint64_t* rs, uint64_t* re, uint32_t* rtext, hipStream_t s);

// Outputs.
// Pack marks of each text into its own word range: words of text t start at
// woff[t]; tfirst/tcount give its blocks.
hipError_t launch_pack_marks(const uint8_t* marked, uint32_t T, const uint64_t* tfirst,
                             const uint64_t* tcount, const uint64_t* woff, uint64_t nwords,
                             uint64_t* words, hipStream_t s);
// Leaves: bytes of every block of the last level, block after block.
hipError_t launch_leaves(const uint8_t* T, const LevelDev& lv, const TextsDev& tx,
                         uint8_t* out, hipStream_t s);

// ---- optional pruning (prune.hip) ----
constexpr uint8_t kPruneNot = 0;       // not a candidate
constexpr uint8_t kPruneOpen = 1;      // candidate, undecided
constexpr uint8_t kPrunePruned = 2;
constexpr uint8_t kPruneKept = 3;      // kept, targets not yet released
constexpr uint8_t kPruneKeptDone = 4;
struct PruneDev {
  LevelDev lv;              // one level in its built (unpruned) layout, runs valid
  TextsDev tx;
  const uint64_t* lm;       // [c] leftmost occurrence of every block on the level
  uint8_t* marked;          // [c] marks; pruned blocks are cleared in place
  uint8_t* tgt;             // [c] zeroed: targeted by a pointer of the level
  uint8_t* state;           // [c] kPrune*
  uint64_t* tinfo;          // [c] a candidate's target block; bit 63: spills into the next
  uint32_t* pending;        // [c] open candidates that target the block
  uint64_t* counters;       // [1] candidates still open after a round
  const uint8_t* cmarked;   // child level's final marks; null when the children are leaves
  uint8_t* cgone;           // [child c] zeroed: set for children of pruned blocks
  const uint64_t* cs;       // [c+1] exclusive scan of child counts
  const uint64_t* tfirst;   // [T] first block of each text on this level
  const uint64_t* ctfirst;  // [T] first block of each text on the child level
  uint32_t* err;            // set to 1 on a broken invariant
};
// targets, candidates and the edges between candidates
hipError_t launch_prune_decide_begin(const PruneDev& d, hipStream_t s);
// one settling round; counters[0] = candidates still open afterwards
hipError_t launch_prune_round(const PruneDev& d, hipStream_t s);
hipError_t launch_prune_apply(const PruneDev& d, hipStream_t s);

struct CompactDev {
  uint64_t c;               // blocks before compaction
  const uint64_t* kidx;     // [c+1] exclusive scan of the keep flags
  const uint64_t* uold;     // [c+1] exclusive scan of the kept-and-unmarked flags
  const uint64_t* st;
  const uint32_t* text;
  const uint8_t* marked;    // may be null (leaf level)
  const uint64_t* lm;       // may be null (leaf level)
  uint64_t* nst;
  uint32_t* ntext;
  uint8_t* nmarked;
  uint64_t* nlm;
  uint64_t* nuoff;          // [kept+1] unmarked ranks of the compacted level
};
// keep[i] = !gone[i]; unmk[i] = kept and unmarked (0 everywhere when marked is null)
hipError_t launch_keep_flags(const uint8_t* gone, const uint8_t* marked, uint64_t c, uint64_t* keep,
                             uint64_t* unmk, hipStream_t s);
hipError_t launch_compact(const CompactDev& d, hipStream_t s);
hipError_t launch_gather_firsts(const uint64_t* kidx, const uint64_t* tfirst, uint32_t T,
                                uint64_t* out, hipStream_t s);

}  // namespace bt
