// The window loop of the probe scans in memory-lean builds (device code shared
// by level.hip and probe_text.hip).
//
// Lean builds keep the 32-bit prefix hashes sampled, Hs[q] = H[pbase + 16 q],
// as they keep the 61-bit ones.  A window's hash from the samples alone costs
// two samples and up to 30 Horner steps, so lane l of a chunk takes the kLeanK
// consecutive window numbers w0 = chunk + kLeanK l .. w0 + kLeanK - 1: it forms
// the first window's hash from the samples and rolls it to the next start with
// the byte that leaves and the byte that enters,
//   h(i+1) = (h(i) - T[i] x^(L-1)) x + T[i+L]   (mod 2^32),
// reading the two runs of bytes with three 8-byte loads each.  The short final
// key of a text (shorter than the main windows) rolls its own hash the same
// way from the same start.
#pragma once
#include "common.hpp"
#include "internal.hpp"
#include "window.hpp"

namespace bt {

constexpr int kLeanK = 16;  // consecutive windows per lane

// Segment holding window number w among segments [lo, hi): the last r there
// with woff[r] <= w (lo when none is).
__device__ __forceinline__ uint64_t segment_in(const uint64_t* __restrict__ woff, uint64_t lo,
                                               uint64_t hi, uint64_t w) {
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) >> 1;
    if (woff[mid] <= w) lo = mid; else hi = mid;
  }
  return lo;
}
__device__ __forceinline__ uint64_t segment_of(const uint64_t* __restrict__ woff, uint64_t R,
                                               uint64_t w) {
  return segment_in(woff, 0, R, w);
}

// One lane's kLeanK windows from w0, whose segments lie in [rlo, rhi) (the
// whole wave calls it: push is wave-wide).  TEXT: segments carry texts (the text table is read).  SALT: the
// text's salt is added to every hash and fingerprint.  on_text(t) runs for the
// first text and whenever the lane moves to another one; test8(hv, ok) tests
// eight salted hashes at once, test1(h) one; push(cand, i, t) takes every
// window slot (cand false where there is no window).
template <bool ODD, bool TEXT, bool SALT, class OnText, class Test8, class Test1, class Push>
__device__ __forceinline__ void lean_chunk(const PhaseArgs& a, const uint64_t* __restrict__ woff,
                                           uint64_t rlo, uint64_t rhi, uint64_t W, uint64_t w0,
                                           OnText on_text, Test8 test8, Test1 test1, Push push) {
  const uint32_t* __restrict__ Hs = a.Hs;
  const uint8_t* __restrict__ T = a.T;
  const uint64_t base = a.pbase, end = a.pend, L = a.Lmain, fmask = a.fpmask;
  const uint32_t x32 = a.x32, x32L = a.x32L, x32Lm1 = a.x32Lm1;
  const auto h32 = [&](uint64_t i) { return h32_at(Hs, T, base, end, x32, i); };

  uint64_t r = segment_in(woff, rlo, rhi, w0);
  uint64_t wo = woff[r], wn = woff[r + 1], rs = a.lv.rs[r], re = a.lv.re[r];
  // lanes past the last window hold no segment: they read no text entry
  uint32_t t = (TEXT && w0 < W) ? a.lv.rtext[r] : 0;
  uint64_t salt = SALT ? a.tx.tsalt[t] : 0;
  on_text(t);
  // the text's short final key, if any: length, position, 32-bit hash, x^oL
  // and x^(oL-1)
  uint64_t oL = 0, opos = 0;
  uint32_t oh = 0, ox = 0, oxm1 = 0;
  const auto load_odd = [&]() {
    oL = a.odd.L[t];
    if (oL) {
      opos = a.odd.pos[t];
      const uint64_t hx = a.odd.h32[t];
      oh = (uint32_t)hx;
      ox = (uint32_t)(hx >> 32);
      oxm1 = ox * a.x32inv;
    }
  };
  if (ODD && w0 < W) load_odd();
  // the short key's 61-bit fingerprint at i, against the key's
  const auto odd61 = [&](uint64_t i) {
    uint64_t g = win61<true>(a, i, oL, a.odd.xp[t]);
    if (SALT) g = add61(g, salt);
    if ((g & fmask) == a.odd.fp[t] && i < a.odd.best[t])
      atomicMin((unsigned long long*)&a.odd.best[t], (unsigned long long)i);
  };

  // every lane's windows inside its segment: straight-line rolling
  {
    const uint64_t wl = w0 + kLeanK - 1;
    const bool lane_ok = wl < wn && rs + (wl - wo) + L <= re;
    if (__ballot(lane_ok) == ~0ull) {
      const uint64_t i0 = rs + (w0 - wo);
      const uint32_t s32 = (uint32_t)salt;
      const uint32_t hA = h32(i0);
      uint64_t olo, ohi;  // the bytes that leave, T[i0 ..]
      bytes16_at(T, end, i0, olo, ohi);
      if (ODD && oL) {
        // the short key first (its windows fit wherever the main ones do,
        // oL < L): a mask of the starts whose 32-bit hash matches, then the
        // rare 61-bit checks
        uint32_t ho = h32(i0 + oL) - hA * ox;
        uint64_t plo, phi;
        bytes16_at(T, end, i0 + oL, plo, phi);
        uint32_t om = 0;
#pragma unroll
        for (int k = 0; k < kLeanK; ++k) {
          if (k) ho = roll32(ho, byte_of16(olo, ohi, k - 1), byte_of16(plo, phi, k - 1), oxm1, x32);
          if (i0 + k < opos && ho + s32 == oh) om |= 1u << k;
        }
        while (om) {
          const int k = __builtin_ctz(om);
          om &= om - 1;
          odd61(i0 + k);
        }
      }
      uint32_t h = h32(i0 + L) - hA * x32L;
      uint64_t ilo, ihi;  // the bytes that enter, T[i0 + L ..]
      bytes16_at(T, end, i0 + L, ilo, ihi);
      // eight windows at a time: roll, test together, queue
#pragma unroll
      for (int k0 = 0; k0 < kLeanK; k0 += 8) {
        uint32_t hv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int kk = k0 + k;
          if (kk) h = roll32(h, byte_of16(olo, ohi, kk - 1), byte_of16(ilo, ihi, kk - 1), x32Lm1, x32);
          hv[k] = h + s32;
        }
        bool ok[8];
        test8(hv, ok);
#pragma unroll
        for (int k = 0; k < 8; ++k) push(ok[k], i0 + k0 + k, t);
      }
      return;
    }
  }

  // per step, following the lane across segment (and text) boundaries: roll
  // while the windows stay consecutive, else start afresh from the samples.
  // pi, opi: start of the hash held plus one, 0 = none (window starts can be
  // 0, so "start + 1 == i" with a sentinel start would wrap onto them)
  uint64_t pi = 0, opi = 0;
  uint32_t h = 0, ho = 0;
  for (int k = 0; k < kLeanK; ++k) {
    const uint64_t w = w0 + (uint64_t)k;
    const bool live = w < W;  // every lane stays in the loop (the queue is wave-wide)
    if (live && w >= wn) {
      do {
        ++r;
        wo = wn;
        wn = woff[r + 1];
      } while (w >= wn);
      rs = a.lv.rs[r];
      re = a.lv.re[r];
      if (TEXT) {
        const uint32_t nt = a.lv.rtext[r];
        if (nt != t) {
          t = nt;
          if (SALT) salt = a.tx.tsalt[t];
          on_text(t);
          if (ODD) {
            load_odd();
            opi = 0;
          }
        }
      }
    }
    const uint64_t i = rs + (w - wo);
    bool cand = false;
    if (live && i + L <= re) {
      h = (pi && i == pi) ? roll32(h, T[i - 1], T[i - 1 + L], x32Lm1, x32)
                          : h32(i + L) - h32(i) * x32L;
      pi = i + 1;
      cand = test1(h + (uint32_t)salt);
    }
    push(cand, i, t);
    if (ODD && live && oL && i + oL <= re && i < opos) {
      ho = (opi && i == opi) ? roll32(ho, T[i - 1], T[i - 1 + oL], oxm1, x32)
                             : h32(i + oL) - h32(i) * ox;
      opi = i + 1;
      if (ho + (uint32_t)salt == oh) odd61(i);
    }
  }
}

}  // namespace bt
