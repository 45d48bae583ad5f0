// Device helpers shared by the probe scans (level.hip, probe_text.hip): the
// table probe, the per-wave candidate queue's constants, wave-level sync.
#pragma once
#include "common.hpp"
#include "internal.hpp"

namespace bt {

// Linear probing from the home slot: the slots up to the first empty one are
// exactly those a key with this fingerprint could occupy.  A slot is 16 bytes
// and eight share a 128-byte line, so a probe that ends near its home slot (the
// usual case at the table's load) reads one line.  Most probes at the deep
// levels, where probes are most numerous, hit a key.
__device__ __forceinline__ void probe(Slot* __restrict__ slots, uint64_t mask, uint64_t fp,
                                      uint64_t i) {
  uint64_t h = slot_of(fp, mask);
  while (true) {
    const Slot s = slots[h];
    if (s.fp == fp) {
      if (i < s.best) atomicMin((unsigned long long*)&slots[h].best, (unsigned long long)i);
      return;
    }
    if (s.fp == kEmpty) return;
    h = (h + 1) & mask;
  }
}


constexpr int kQueue = 128;  // entries per wave (< 64 pending + up to 64 new)

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Queue entries pack a window start (below 2^40) and its text (below 2^24).
constexpr int kQPosBits = 40;
constexpr uint64_t kQPosMask = (1ull << kQPosBits) - 1;

}  // namespace bt
