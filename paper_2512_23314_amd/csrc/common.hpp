// Device-side helpers shared by the HIP kernels of libbt (gfx950 only).
//
// Arithmetic is exact integer arithmetic modulo the Mersenne prime
// q = 2^61 - 1, which is the Karp-Rabin modulus of this library (Section 2 of
// the paper allows any q in Theta(n^c); 2^61-1 keeps collision odds per
// comparison below L / 2^61 and reduces with shifts and adds).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bt {

constexpr uint64_t kP61 = 0x1FFFFFFFFFFFFFFFull;
constexpr uint64_t kEmpty = ~0ull;          // empty hash slot / "no position"
constexpr uint32_t kNoKey = 0xFFFFFFFFu;    // block has no key in this phase
constexpr uint32_t kOddKey = 0xFFFFFFFEu;   // key of non-standard length (text tail)
// The key's string is known to occur earlier (from the level above); it is not
// inserted, and its leftmost occurrence is recorded as "before its start".
constexpr uint32_t kCopyKey = 0xFFFFFFFDu;
constexpr uint64_t kWeakMask = 0xFFFull;    // BT_DBG_WEAK_HASH truncation

// (a b + c) mod (2^61 - 1) for a, b, c < 2^61.  The product is
// p11 2^64 + mid 2^32 + p00 from four 32 x 32-bit products (no 64-bit high
// multiply); with 2^64 = 8 and 2^61 = 1 (mod q) every part folds to a term
// below 2^61, the sum stays below 2^63, and one more fold and one conditional
// subtraction give the residue.
__device__ __forceinline__ uint64_t mad61(uint64_t a, uint64_t b, uint64_t c) {
  const uint64_t a0 = (uint32_t)a, a1 = a >> 32, b0 = (uint32_t)b, b1 = b >> 32;
  const uint64_t p00 = a0 * b0;
  const uint64_t mid = a0 * b1 + a1 * b0;  // < 2^62
  const uint64_t p11 = a1 * b1;            // < 2^58
  uint64_t s = (p11 << 3) + (mid >> 29) + ((mid & ((1ull << 29) - 1)) << 32) + (p00 >> 61) +
               (p00 & kP61) + c;
  s = (s & kP61) + (s >> 61);
  return s >= kP61 ? s - kP61 : s;
}
// a * b mod (2^61 - 1) for a, b < 2^61.
__device__ __forceinline__ uint64_t mul61(uint64_t a, uint64_t b) { return mad61(a, b, 0); }
__device__ __forceinline__ uint64_t add61(uint64_t a, uint64_t b) {
  const uint64_t r = a + b;
  return r >= kP61 ? r - kP61 : r;
}
__device__ __forceinline__ uint64_t sub61(uint64_t a, uint64_t b) {
  return a >= b ? a - b : a + kP61 - b;
}
__device__ inline uint64_t pow61(uint64_t x, uint64_t e) {
  uint64_t r = 1;
  while (e) {
    if (e & 1) r = mul61(r, x);
    x = mul61(x, x);
    e >>= 1;
  }
  return r;
}

// Fingerprint of T[i .. i+L) from prefix fingerprints: P[i+L] - P[i] * x^L.
__device__ __forceinline__ uint64_t window_fp(const uint64_t* __restrict__ P, uint64_t i,
                                              uint64_t L, uint64_t xL) {
  return sub61(P[i + L], mul61(P[i], xL));
}

// Final key of a window: add the per-text salt (batched builds keep texts
// apart), then apply the debug truncation mask (all ones normally).
__device__ __forceinline__ uint64_t finish_fp(uint64_t fp, uint64_t salt, uint64_t mask) {
  return add61(fp, salt) & mask;
}

// Home slot of a fingerprint in a power-of-two open-addressing table.
__device__ __forceinline__ uint64_t slot_of(uint64_t fp, uint64_t mask) {
  return (fp ^ (fp >> 29) ^ (fp >> 47)) & mask;
}

// The two bits of a fingerprint in a key filter of 2^bits bits.
__device__ __forceinline__ uint64_t filter_bit(uint64_t fp, uint32_t bits) {
  return (fp ^ (fp >> 31)) & ((1ull << bits) - 1);
}
__device__ __forceinline__ uint64_t filter_bit2(uint64_t fp, uint32_t bits) {
  return ((fp >> 17) ^ (fp >> 41) ^ (fp * 0x9E3779B1ull >> 20)) & ((1ull << bits) - 1);
}

// The two bits of a 32-bit window hash (mod 2^32 polynomial hash, whose high
// bits depend on every byte) in a filter of 2^bits bits.
__device__ __forceinline__ uint32_t filter_bit32(uint32_t h, uint32_t bits) {
  return h >> (32 - bits);
}
__device__ __forceinline__ uint32_t filter_bit32b(uint32_t h, uint32_t bits) {
  return (h * 0x9E3779B1u) >> (32 - bits);
}

// Second (global, L2-resident) filter of a 32-bit window hash: blocked, three
// bits in one 64-bit word, so that a test is one load.  The word and the bit
// positions come from multiplicative hashes with their own odd constants,
// unrelated to the bits the LDS filter takes.  words_log2 = log2(64-bit words).
__device__ __forceinline__ uint32_t filter2_word(uint32_t h, uint32_t words_log2) {
  return (h * 0x6F4F2A35u) >> (32 - words_log2);
}
__device__ __forceinline__ uint64_t filter2_mask(uint32_t h) {
  const uint32_t m = h * 0xD35A2D97u;
  return (1ull << (m >> 26)) | (1ull << ((m >> 20) & 63)) | (1ull << ((m >> 14) & 63));
}

// Text-local filter of a 32-bit window hash (batches): blocked, three bits in
// one 32-bit word, so that a test is one 4-byte load.  words_log2 (>= 3) =
// log2(32-bit words); word and bits come from multiplicative hashes with their
// own odd constants.
__device__ __forceinline__ uint32_t tfilter_word(uint32_t h, uint32_t words_log2) {
  return (h * 0x7FEB352Du) >> (32 - words_log2);
}
__device__ __forceinline__ uint32_t tfilter_mask(uint32_t h) {
  const uint32_t m = h * 0x846CA68Bu;
  return (1u << (m >> 27)) | (1u << ((m >> 22) & 31)) | (1u << ((m >> 17) & 31));
}

// Filter bit of a string's first eight bytes (lo = bytes 0..3, hi = bytes
// 4..7, little endian) in a filter of 2^bits bits: equal strings of length 8 or
// more share it.  The top bits of each product depend on every bit of its word.
__device__ __forceinline__ uint32_t prefix8_bit(uint32_t lo, uint32_t hi, uint32_t bits) {
  return ((lo * 0x9E3779B1u) ^ (hi * 0x85EBCA77u)) >> (32 - bits);
}

// P[i] from prefix fingerprints sampled every 2^sh positions (Ps[q] = P[base +
// 2^sh q], sh <= 4): the sample at or below i, then Horner's rule over the
// bytes between.  The up to 15 bytes come from three aligned 8-byte loads
// issued together (one dependent byte load per step would wait a memory round
// trip each), when the words lie inside the text [.., end); else byte by byte.
__device__ __forceinline__ uint64_t prefix_at(const uint64_t* __restrict__ Ps,
                                              const uint8_t* __restrict__ T, uint64_t base,
                                              uint64_t end, uint64_t x, uint64_t i, uint32_t sh) {
  const uint64_t r = i - base;
  const uint32_t m = (uint32_t)(r & ((1u << sh) - 1));
  uint64_t v = Ps[r >> sh];
  if (!m) return v;
  const uint64_t j0 = i - m;
  if (j0 + 24 <= end) {
    // the words at the 8-byte boundary at or below T + j0 cover its 16 bytes
    // (and start no lower than the allocation, whose base is aligned)
    const uintptr_t ad = reinterpret_cast<uintptr_t>(T + j0);
    const uint64_t* wp = reinterpret_cast<const uint64_t*>(ad & ~(uintptr_t)7);
    const uint32_t sh = (uint32_t)(ad & 7) * 8;
    const uint64_t w0 = wp[0], w1 = wp[1], w2 = wp[2];
    const uint64_t lo = sh ? (w0 >> sh) | (w1 << (64 - sh)) : w0;  // bytes j0 .. j0+7
    const uint64_t hi = sh ? (w1 >> sh) | (w2 << (64 - sh)) : w1;  // bytes j0+8 .. j0+15
#pragma unroll
    for (uint32_t k = 0; k < 15; ++k) {
      if (k >= m) break;
      const uint64_t b = ((k < 8 ? lo : hi) >> (8 * (k & 7))) & 0xFF;
      v = mad61(v, x, b);
    }
    return v;
  }
  for (uint64_t j = j0; j < i; ++j) v = mad61(v, x, T[j]);
  return v;
}

// The 15 bytes T[j0 .. j0 + 15) as two words (lo: bytes 0..7, hi: bytes 8..14
// and one more), from three aligned 8-byte loads issued together when the words
// lie inside [.., end); else byte by byte (bytes at or past end read as 0).
__device__ __forceinline__ void bytes16_at(const uint8_t* __restrict__ T, uint64_t end, uint64_t j0,
                                           uint64_t& lo, uint64_t& hi) {
  if (j0 + 24 <= end) {
    const uintptr_t ad = reinterpret_cast<uintptr_t>(T + j0);
    const uint64_t* wp = reinterpret_cast<const uint64_t*>(ad & ~(uintptr_t)7);
    const uint32_t sh = (uint32_t)(ad & 7) * 8;
    const uint64_t w0 = wp[0], w1 = wp[1], w2 = wp[2];
    lo = sh ? (w0 >> sh) | (w1 << (64 - sh)) : w0;
    hi = sh ? (w1 >> sh) | (w2 << (64 - sh)) : w1;
    return;
  }
  lo = hi = 0;
  for (uint32_t k = 0; k < 16 && j0 + k < end; ++k)
    (k < 8 ? lo : hi) |= (uint64_t)T[j0 + k] << (8 * (k & 7));
}

// H[i] from 32-bit prefix hashes sampled every 16 positions (Hs[q] = H[base +
// 16 q], H[j+1] = H[j] x32 + T[j] mod 2^32): the sample at or below i, then
// Horner's rule over the at most 15 bytes between (i < end).
__device__ __forceinline__ uint32_t h32_at(const uint32_t* __restrict__ Hs,
                                           const uint8_t* __restrict__ T, uint64_t base,
                                           uint64_t end, uint32_t x32, uint64_t i) {
  const uint64_t r = i - base;
  const uint32_t m = (uint32_t)(r & 15);
  uint32_t v = Hs[r >> 4];
  if (!m) return v;
  uint64_t lo, hi;
  bytes16_at(T, end, i - m, lo, hi);
#pragma unroll
  for (uint32_t k = 0; k < 15; ++k) {
    if (k >= m) break;
    v = v * x32 + (uint32_t)(((k < 8 ? lo : hi) >> (8 * (k & 7))) & 0xFF);
  }
  return v;
}

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Relaxed device-scope store: the word carries its own payload, so no other
// memory needs ordering with it (a release here would write back the L2).
__device__ __forceinline__ void st_relaxed(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// v of lane src (every lane of the wave takes part), in two 32-bit halves.
__device__ __forceinline__ uint64_t shfl64(uint64_t v, uint32_t src) {
  const uint32_t lo = __shfl((uint32_t)v, (int)src), hi = __shfl((uint32_t)(v >> 32), (int)src);
  return ((uint64_t)hi << 32) | lo;
}

// Sum of a 64-lane wave under add61.
__device__ __forceinline__ uint64_t wave_sum61(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = add61(v, __shfl_xor(v, d));
  return v;
}

// 16 bytes from an arbitrary byte address (unaligned global load).
__device__ __forceinline__ uint4 load16(const uint8_t* p) {
  uint4 v;
  __builtin_memcpy(&v, p, 16);
  return v;
}

}  // namespace bt
