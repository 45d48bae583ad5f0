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
  // rank/select support (see query.hip)
  const uint64_t* cnt;     // [c * S]: occurrences of each symbol before the block start
  const uint64_t* pcnt;    // [u * S]: occurrences of each symbol in the target pair
                           //           before the source position
};

struct QTree {
  const QLevel* lv;        // h entries
  uint32_t h;
  uint32_t tau;
  uint64_t n;
  const uint8_t* leaves;   // leaf block j at j * leaf_len
  uint64_t leaf_len;
  const int16_t* sym;      // byte -> dense symbol (-1 = absent)
  uint32_t S;              // dense alphabet size
  const uint64_t* leafcnt; // [c_h * S] occurrences before each leaf block
};

hipError_t launch_access(QTree t, const uint64_t* pos, uint64_t m, uint8_t* out, uint32_t* bad,
                         hipStream_t s);
hipError_t launch_rank(QTree t, const uint8_t* cs, const uint64_t* pos, uint64_t m, uint64_t* out,
                       hipStream_t s);
hipError_t launch_select(QTree t, const uint8_t* cs, const uint64_t* ks, uint64_t m,
                         uint64_t* out, hipStream_t s);

// auxiliary kernels used by the build
hipError_t launch_histogram(const uint8_t* T, uint64_t n, uint64_t* hist, hipStream_t s);
hipError_t launch_last_block_len(const LevelDev& lv, const TextsDev& tx, const uint64_t* tfirst,
                                 const uint64_t* tcount, uint64_t* out, hipStream_t s);
hipError_t launch_text_deltas(const uint64_t* scanned, const uint64_t* tfirst,
                              const uint64_t* tcount, uint32_t T, uint64_t* out, hipStream_t s);
hipError_t launch_word_pop(const uint64_t* words, uint64_t nwords, uint64_t* out, hipStream_t s);
hipError_t launch_word_rank(const uint64_t* scanned, uint32_t T, const uint64_t* woff,
                            uint64_t nwords, uint64_t* wrank, hipStream_t s);

}  // namespace bt
