// Query-side view of a tree (device data) and the query/auxiliary launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace bt {

constexpr uint64_t kP61Host = 0x1FFFFFFFFFFFFFFFull;

// One level of a finished tree, as the query kernels read it.
struct QLevel {
  uint64_t b;              // block length
  uint64_t c;              // blocks
  const uint64_t* words;   // marks, ceil(c/64) words, LSB first
  const uint64_t* wrank;   // marks before each word (within this tree)
  const uint64_t* pb;      // pointer block (level-local), one per unmarked block
  const uint64_t* po;      // pointer offset
  // rank/select support (rank.hip); all null when the tree was built without it
  const uint32_t* acnt;    // [c * S]: occurrences of each symbol before the block
                           //          (from the text's start), or null on a
                           //          relative level:
  const uint8_t* qc;       // [c * S]: occurrences inside the parent before the
                           //          block, qw bytes each
  const uint8_t* pc;       // [u * S]: occurrences between the target block's start
                           //          and the source position, pw bytes each
  const uint32_t* msel;    // [marked blocks]: index of each marked block (internal
                           //          levels; the parent of child j is msel[j / tau])
  const uint64_t* st;      // [c] block starts (positions in the build's buffer)
  uint32_t qw, pw;         // widths in bytes (1, 2 or 4)
};

struct QTree {
  const QLevel* lv;        // h entries
  uint32_t h;
  uint32_t tau;
  uint64_t n;
  const uint8_t* leaves;   // leaf block j at j * leaf_len
  uint64_t leaf_len;
  const int16_t* sym;      // byte -> dense symbol (-1 = absent), 256 entries
  uint32_t S;              // dense alphabet size
  const uint64_t* total;   // [S] occurrences in the whole text
  uint64_t tstart;         // position of the text in the build's buffer
};

// Rank support construction.
constexpr uint64_t kRankQ = 1024;  // sampling interval of the count table
struct RankCtx {
  const uint8_t* T;        // the build's buffer
  uint64_t o0;             // first position covered by the table
  const uint64_t* G;       // [(K + 1) * S] counts before each sampled position
  uint32_t S;
  const uint8_t* byte_of;  // [S] dense symbol -> byte
};
hipError_t build_count_table(const uint8_t* T, uint64_t o0, uint64_t N, const int16_t* sym,
                             uint32_t S, uint32_t* H, uint64_t* B, uint64_t* G, hipStream_t s);
hipError_t launch_text_rank_counts(const RankCtx& rc, const TextsDev& tx, uint64_t* Rt,
                                   uint64_t* Rtot, hipStream_t s);
hipError_t launch_block_rank_counts(const RankCtx& rc, const uint64_t* st, const uint32_t* text,
                                    uint64_t c, const uint64_t* Rt, uint32_t* cnt, hipStream_t s);
hipError_t launch_pointer_rank_counts(const RankCtx& rc, const uint64_t* st, const uint32_t* text,
                                      const uint8_t* marked, uint64_t c, const uint64_t* uoff,
                                      const uint64_t* tfirst, const uint64_t* pb,
                                      const uint64_t* po, const uint64_t* Rt, const uint32_t* cnt,
                                      uint8_t* pcnt, uint32_t pw, hipStream_t s);
// Relative counts of a level from its absolute ones A (u32, from the text's
// start), qw bytes each.
hipError_t launch_relative_counts(const uint32_t* A, uint64_t c, uint32_t S, const uint32_t* text,
                                  const uint64_t* tfirst, uint32_t tau, uint8_t* q, uint32_t qw,
                                  hipStream_t s);
// Copies of absolute rows: ent holds E triples (first row, rows, destination row).
hipError_t launch_root_rows(const uint32_t* A, uint32_t S, const uint64_t* ent, uint32_t E,
                            uint32_t* out, hipStream_t s);
hipError_t launch_marked_index(const uint8_t* marked, const uint64_t* uoff, uint64_t c,
                               const uint32_t* text, const uint64_t* tfirst, uint32_t* msel,
                               hipStream_t s);
// Bytes of a counter that holds values up to vmax: 1, 2 or 4.
inline uint32_t counter_width(uint64_t vmax) { return vmax <= 0xFF ? 1u : vmax <= 0xFFFF ? 2u : 4u; }

hipError_t launch_access(QTree t, const uint64_t* pos, uint64_t m, uint8_t* out, uint32_t* bad,
                         hipStream_t s);
hipError_t launch_rank(QTree t, const uint8_t* cs, const uint64_t* pos, uint64_t m, uint64_t* out,
                       hipStream_t s);
hipError_t launch_select(QTree t, const uint8_t* cs, const uint64_t* ks, uint64_t m,
                         uint64_t* out, hipStream_t s);
// rank on an empty text: 0 for position 0, UINT64_MAX otherwise
hipError_t launch_rank_empty(const uint64_t* pos, uint64_t m, uint64_t* out, hipStream_t s);

// auxiliary kernels used by the build
// Which byte values occur in T[0..n): bit c of the 256-bit set `seen` (eight
// words, zeroed by the caller) is set when byte value c occurs.
hipError_t launch_byte_presence(const uint8_t* T, uint64_t n, uint32_t* seen, hipStream_t s);
hipError_t launch_last_block_len(const LevelDev& lv, const TextsDev& tx, const uint64_t* tfirst,
                                 const uint64_t* tcount, uint64_t* out, hipStream_t s);
hipError_t launch_text_deltas(const uint64_t* scanned, const uint64_t* tfirst,
                              const uint64_t* tcount, uint32_t T, uint64_t* out, hipStream_t s);
hipError_t launch_word_pop(const uint64_t* words, uint64_t nwords, uint64_t* out, hipStream_t s);
hipError_t launch_word_rank(const uint64_t* scanned, uint32_t T, const uint64_t* woff,
                            uint64_t nwords, uint64_t* wrank, hipStream_t s);

}  // namespace bt
