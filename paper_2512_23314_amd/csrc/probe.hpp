// Device helpers shared by the probe scans (level.hip, probe_text.hip): the
// table probe, the per-wave candidate queue's constants, wave-level sync.
#pragma once
#include "common.hpp"
#include "internal.hpp"

namespace bt {

// Linear probing over the tag array, one aligned group of eight tags per load:
// the slots from the home slot up to the first empty one are exactly those a
// key with this fingerprint could occupy; only those whose tag matches are read.
__device__ __forceinline__ void probe(Slot* __restrict__ slots, const uint8_t* __restrict__ tags,
                                      uint64_t mask, uint64_t fp, uint64_t i) {
  constexpr uint64_t kLo7 = 0x7F7F7F7F7F7F7F7Full;
  const uint64_t h = slot_of(fp, mask);
  const uint64_t tb = 0x0101010101010101ull * tag_of(fp);
  uint64_t g = h >> 3;
  uint64_t valid = ~0ull << (8 * (h & 7));  // bytes at or after the home slot
  while (true) {
    const uint64_t w = *reinterpret_cast<const uint64_t*>(tags + 8 * g);
    // bit 8k+7 set exactly where byte k is zero (empty) / equals the tag
    const uint64_t emp = ~(((w & kLo7) + kLo7) | w | kLo7) & valid;
    const uint64_t x = w ^ tb;
    uint64_t mat = ~(((x & kLo7) + kLo7) | x | kLo7) & valid;
    if (emp) mat &= (emp & (0 - emp)) - 1;  // matches before the first empty slot
    while (mat) {
      const uint64_t j = 8 * g + (__builtin_ctzll(mat) >> 3);
      const Slot s = slots[j];
      if (s.fp == fp) {
        if (i < s.best) atomicMin((unsigned long long*)&slots[j].best, (unsigned long long)i);
        return;
      }
      mat &= mat - 1;
    }
    if (emp) return;
    g = (g + 1) & (mask >> 3);
    valid = ~0ull;
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
