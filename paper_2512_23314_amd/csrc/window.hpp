// Window fingerprints of a phase (device code shared by the scan kernels).
#pragma once
#include "common.hpp"
#include "internal.hpp"

namespace bt {

// P[i+L] - P[i] x^L from dense prefix fingerprints, or (LEAN) from the samples
// of a memory-lean build.
template <bool LEAN>
__device__ __forceinline__ uint64_t win61(const PhaseArgs& a, uint64_t i, uint64_t L, uint64_t xL) {
  if (LEAN)
    return sub61(prefix_at(a.Ps, a.T, a.pbase, a.pend, a.x, i + L),
                 mul61(prefix_at(a.Ps, a.T, a.pbase, a.pend, a.x, i), xL));
  return sub61(a.P[i + L], mul61(a.P[i], xL));
}
__device__ __forceinline__ uint64_t win61_any(const PhaseArgs& a, uint64_t i, uint64_t L,
                                              uint64_t xL) {
  return a.P ? win61<false>(a, i, L, xL) : win61<true>(a, i, L, xL);
}

}  // namespace bt
