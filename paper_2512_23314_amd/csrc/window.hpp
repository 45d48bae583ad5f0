// Window fingerprints of a phase (device code shared by the scan kernels).
#pragma once
#include "common.hpp"
#include "internal.hpp"

namespace bt {

// P[i+L] - P[i] x^L from dense prefix fingerprints, or (LEAN) from samples.
template <bool LEAN>
__device__ __forceinline__ uint64_t win61(const PhaseArgs& a, uint64_t i, uint64_t L, uint64_t xL) {
  if (LEAN)
    return sub61(prefix_at(a.Ps, a.T, a.pbase, a.pend, a.x, i + L, a.pshift),
                 mul61(prefix_at(a.Ps, a.T, a.pbase, a.pend, a.x, i, a.pshift), xL));
  return sub61(a.P[i + L], mul61(a.P[i], xL));
}
__device__ __forceinline__ uint64_t win61_any(const PhaseArgs& a, uint64_t i, uint64_t L,
                                              uint64_t xL) {
  return a.P ? win61<false>(a, i, L, xL) : win61<true>(a, i, L, xL);
}

// The 32-bit hash H[i+L] - H[i] xL (mod 2^32) of a window, from dense prefix
// hashes or from the samples of a memory-lean build.
__device__ __forceinline__ uint32_t win32_any(const PhaseArgs& a, uint64_t i, uint64_t L,
                                              uint32_t xL) {
  if (a.P32) return a.P32[i + L] - a.P32[i] * xL;
  return h32_at(a.Hs, a.T, a.pbase, a.pend, a.x32, i + L) -
         h32_at(a.Hs, a.T, a.pbase, a.pend, a.x32, i) * xL;
}

// Lean scans roll a window's 32-bit hash to the next start:
// h(i+1) = (h(i) - T[i] x^(L-1)) x + T[i+L] (mod 2^32).
__device__ __forceinline__ uint32_t roll32(uint32_t h, uint32_t out, uint32_t in, uint32_t xLm1,
                                           uint32_t x) {
  return (h - out * xLm1) * x + in;
}

// Byte k (0..15) of the pair of words bytes16_at returns.
__device__ __forceinline__ uint32_t byte_of16(uint64_t lo, uint64_t hi, int k) {
  return (uint32_t)(((k < 8 ? lo : hi) >> (8 * (k & 7))) & 0xFF);
}

}  // namespace bt
