// One level of block-tree construction (Section 4.1): both phases, the split
// into the next level, and the level's outputs.
//
// Phase 1 (a3-a5): the key of every pair of consecutive blocks goes into an
// open-addressing table; every window of length 2b inside a run of consecutive
// blocks is fingerprinted from the prefix fingerprints and probed; a hit at
// position i lowers the slot's smallest position with atomicMin.  Phase 2
// (a6-a7) does the same for unmarked blocks with windows of length b.  Keys
// with the same fingerprint share a slot, so a slot's minimum is the leftmost
// position with that fingerprint; each key then compares its bytes with that
// position (a4 verification).  A mismatch -- a fingerprint collision -- sends
// the key to an exact fallback scan that walks the text from just past the
// false hit and verifies every further hit, so the result is the leftmost
// occurrence whatever the hash does.
//
// Only windows inside runs are scanned: for tau >= 2 the leftmost occurrence in
// T of any string no longer than b_{l-1} lies inside a run of level l (it is
// covered by two consecutive marked blocks of level l-1, whose children are
// present), so "leftmost on this level" and "leftmost in T" coincide.
#include "common.hpp"
#include "internal.hpp"
#include "lean.hpp"
#include "probe.hpp"
#include "window.hpp"

namespace bt {

static unsigned grid_for(uint64_t n, unsigned threads, unsigned cap = 8192) {
  uint64_t g = (n + threads - 1) / threads;
  if (g == 0) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

#define GRID_STRIDE(i, n)                                                        \
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
       i += (uint64_t)gridDim.x * blockDim.x)

__device__ __forceinline__ uint64_t block_len(const LevelDev& lv, const TextsDev& tx,
                                              uint64_t j) {
  const uint64_t st = lv.st[j];
  const uint64_t te = tx.tend[lv.text[j]];
  return te - st < lv.b ? te - st : lv.b;
}

// ---------------------------------------------------------------- keys (a3, a6)

// The key at st (at least 8 bytes long) in the byte scan's prefix filter.
__device__ __forceinline__ void set_prefix_bit(const PhaseArgs& a, uint64_t st) {
  uint32_t lo = 0, hi = 0;
  for (int k = 0; k < 4; ++k) {
    lo |= (uint32_t)a.T[st + k] << (8 * k);
    hi |= (uint32_t)a.T[st + 4 + k] << (8 * k);
  }
  const uint32_t bit = prefix8_bit(lo, hi, a.bfilt_bits);
  atomicOr(&a.bfilt[bit >> 5], 1u << (bit & 31));
}

// Profiling: add a per-thread count to *p, one atomic per wave.
__device__ __forceinline__ void wave_count(uint64_t* p, uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd((unsigned long long*)p, (unsigned long long)v);
}

__global__ void k_keys(PhaseArgs a) {
  const LevelDev lv = a.lv;
  uint64_t inserted = 0;
  GRID_STRIDE(j, lv.c) {
    const uint32_t t = lv.text[j];
    const uint64_t st = lv.st[j];
    const uint64_t len = block_len(lv, a.tx, j);
    uint64_t L = 0;
    bool valid;
    if (a.phase == 1) {
      valid = (j + 1 < lv.c) && lv.run[j + 1] == lv.run[j];
      if (valid) L = len + block_len(lv, a.tx, j + 1);
    } else {
      valid = a.all_blocks || !a.marked[j];
      L = len;
    }
    if (!valid) {
      a.k.slot[j] = kNoKey;
      continue;
    }
    if (a.cflag) {
      // Strings inside a parent region that occurs earlier occur earlier too:
      // a pair window of length 2b <= b_parent starting in a parent whose pair
      // with the next parent occurs earlier, or lying inside a parent that
      // occurs earlier (itself, or as part of its pair with the previous one).
      // Marks and facts only need "before its start" for these; phase 2 needs
      // exact positions for unmarked blocks, and for all blocks when pruning.
      const uint8_t f = a.cflag[j];
      const bool copy = (a.phase == 1)
                            ? ((f & kSkipCross) || ((f & kSkipInterior) && !(f & kLastChild)))
                            : (!a.exact_all && a.marked[j] && (f & (kSkipCross | kSkipInterior)));
      if (copy) {
        a.k.slot[j] = kCopyKey;
        a.k.lm[j] = st - 1;
        continue;
      }
    }
    ++inserted;
    const uint64_t xp = (L == a.Lmain) ? a.xLmain : pow61(a.x, L);
    const uint64_t fp = finish_fp(win61_any(a, st, L, xp), a.tx.tsalt[t], a.fpmask);
    a.k.fp[j] = fp;
    a.k.len[j] = L;
    // (a flag: written once, not by every key of the text into one word)
    if (!a.odd.nkeys[t]) a.odd.nkeys[t] = 1;
    if (L == a.Lmain) {
      uint64_t h = slot_of(fp, a.tab.mask);
      while (true) {
        const uint64_t prev = atomicCAS((unsigned long long*)&a.tab.slots[h].fp,
                                        (unsigned long long)kEmpty, (unsigned long long)fp);
        if (prev == kEmpty || prev == fp) break;
        h = (h + 1) & a.tab.mask;
      }
      a.k.slot[j] = (uint32_t)h;
      atomicMin((unsigned long long*)&a.tab.slots[h].best, (unsigned long long)st);
      if (a.tf_words) {
        // text-local filter: this text's keys only
        const uint32_t h = win32_any(a, st, L, a.x32L) + (uint32_t)a.tx.tsalt[t];
        atomicOr(a.tf_words + a.tf_off[t] + tfilter_word(h, a.tf_wl[t]), tfilter_mask(h));
      }
      if (a.filt_bits) {
        uint64_t f1, f2;
        if (a.pre32) {
          const uint32_t h = win32_any(a, st, L, a.x32L) + (uint32_t)a.tx.tsalt[t];
          f1 = filter_bit32(h, a.filt_bits);
          f2 = filter_bit32b(h, a.filt_bits);
          if (a.filt2_words)
            atomicOr(reinterpret_cast<unsigned long long*>(a.filt2) + filter2_word(h, a.filt2_words),
                     (unsigned long long)filter2_mask(h));
        } else {
          f1 = filter_bit(fp, a.filt_bits);
          f2 = filter_bit2(fp, a.filt_bits);
        }
        atomicOr(&a.filt[f1 >> 5], 1u << (f1 & 31));
        if (a.filt_two) atomicOr(&a.filt[f2 >> 5], 1u << (f2 & 31));
      }
      if (a.bfilt_bits) set_prefix_bit(a, st);
    } else {
      // the one key of this text that ends at the text's end with a short block
      a.k.slot[j] = kOddKey;
      a.odd.L[t] = L;
      a.odd.xp[t] = xp;
      a.odd.fp[t] = fp;
      a.odd.pos[t] = st;
      a.odd.best[t] = st;
      uint32_t x32p = 1, base = a.x32;  // x32^L
      for (uint64_t e = L; e; e >>= 1) {
        if (e & 1) x32p *= base;
        base *= base;
      }
      const uint32_t h = win32_any(a, st, L, x32p) + (uint32_t)a.tx.tsalt[t];
      a.odd.h32[t] = (uint64_t)h | ((uint64_t)x32p << 32);
      if (a.bfilt_bits) set_prefix_bit(a, st);
    }
  }
  if (a.pc) wave_count(a.pc + kPcKeys, inserted);
}

hipError_t launch_keys(const PhaseArgs& a, hipStream_t s) {
  k_keys<<<grid_for(a.lv.c, 256), 256, 0, s>>>(a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- scan segments
//
// The probe scan walks "segments": ranges of window starts, each inside one run.
// A window whose content also occurs earlier can never be the leftmost
// occurrence of anything, so the previous level's results prune segments.  For
// a marked parent block P (all windows of this level start inside some parent):
//   - if the pair (P, P+1) has an earlier occurrence, every window starting in
//     P lies inside a copy of it (windows are at most one parent long);
//   - if the pair (P-1, P) has an earlier occurrence, or P itself does, every
//     window that ends inside P is a copy.
// Entries describe parents (or whole runs where there is no parent level) as
// [a, e) plus these two facts; per phase they become segments.

// Entries from runs: the whole run, nothing skipped.
__global__ void k_entries_from_runs(LevelDev lv, uint64_t* ea, uint64_t* ee, uint8_t* ef,
                                    uint32_t* erun) {
  GRID_STRIDE(r, lv.R) {
    ea[r] = lv.rs[r];
    ee[r] = lv.re[r];
    ef[r] = 0;
    erun[r] = (uint32_t)r;
  }
}

hipError_t launch_entries_from_runs(const LevelDev& lv, uint64_t* ea, uint64_t* ee, uint8_t* ef,
                                    uint32_t* erun, hipStream_t s) {
  if (!lv.R) return hipSuccess;
  k_entries_from_runs<<<grid_for(lv.R, 256), 256, 0, s>>>(lv, ea, ee, ef, erun);
  return hipGetLastError();
}

// Pair facts after phase 1: bit 0 of pf[j] = the pair (j, j+1) occurs earlier.
__global__ void k_pair_facts(PhaseArgs a, uint8_t* pf) {
  GRID_STRIDE(j, a.lv.c) {
    pf[j] = (a.k.slot[j] != kNoKey && a.k.lm[j] < a.lv.st[j]) ? 1 : 0;
  }
}

hipError_t launch_pair_facts(const PhaseArgs& a, uint8_t* pf, hipStream_t s) {
  k_pair_facts<<<grid_for(a.lv.c, 256), 256, 0, s>>>(a, pf);
  return hipGetLastError();
}

// Block facts after a phase 2 over all blocks: bit 1 = block j occurs earlier.
__global__ void k_block_facts(PhaseArgs a, uint8_t* pf) {
  GRID_STRIDE(j, a.lv.c) {
    if (a.k.slot[j] != kNoKey && a.k.lm[j] < a.lv.st[j]) pf[j] |= 2;
  }
}

hipError_t launch_block_facts(const PhaseArgs& a, uint8_t* pf, hipStream_t s) {
  k_block_facts<<<grid_for(a.lv.c, 256), 256, 0, s>>>(a, pf);
  return hipGetLastError();
}

// Entries of the next level: one per marked block P of this level (in order;
// its children start at next index ntfirst[t] + cs[P] - cs[tfirst[t]]), then
// one per entering text (whole text, nothing skipped).
__global__ void k_entries_from_parents(LevelDev lv, TextsDev tx, const uint8_t* marked,
                                       const uint8_t* pf, const uint64_t* uoff, const uint64_t* cs,
                                       const uint64_t* tfirst, const uint64_t* ntfirst,
                                       uint64_t* ea, uint64_t* ee, uint8_t* ef, uint64_t* echild) {
  GRID_STRIDE(P, lv.c) {
    if (!marked[P]) continue;
    const uint64_t k = P - uoff[P];
    const uint32_t t = lv.text[P];
    const uint64_t st = lv.st[P], te = tx.tend[t];
    ea[k] = st;
    ee[k] = st + (te - st < lv.b ? te - st : lv.b);
    uint8_t f = 0;
    if (pf[P] & 1) f |= kSkipCross;
    if ((pf[P] & 2) || (P > 0 && (pf[P - 1] & 1))) f |= kSkipInterior;
    ef[k] = f;
    echild[k] = ntfirst[t] + (cs[P] - cs[tfirst[t]]);
  }
}

__global__ void k_entries_entering(const uint32_t* ids, uint32_t E, TextsDev tx, uint64_t base,
                                   const uint64_t* ntfirst, uint64_t* ea, uint64_t* ee,
                                   uint8_t* ef, uint64_t* echild) {
  GRID_STRIDE(k, E) {
    const uint32_t t = ids[k];
    ea[base + k] = tx.tstart[t];
    ee[base + k] = tx.tend[t];
    ef[base + k] = 0;
    echild[base + k] = ntfirst[t];
  }
}

hipError_t launch_entries_next(const LevelDev& lv, const TextsDev& tx, const uint8_t* marked,
                               const uint8_t* pf, const uint64_t* uoff, const uint64_t* cs,
                               const uint64_t* tfirst, const uint64_t* ntfirst, uint64_t nmarked,
                               const uint32_t* ids, uint32_t E, uint64_t* ea, uint64_t* ee,
                               uint8_t* ef, uint64_t* echild, hipStream_t s) {
  if (lv.c)
    k_entries_from_parents<<<grid_for(lv.c, 256), 256, 0, s>>>(lv, tx, marked, pf, uoff, cs, tfirst,
                                                               ntfirst, ea, ee, ef, echild);
  if (E)
    k_entries_entering<<<grid_for(E, 256), 256, 0, s>>>(ids, E, tx, nmarked, ntfirst, ea, ee, ef,
                                                          echild);
  return hipGetLastError();
}

__global__ void k_child_flags(SegDev sg, uint64_t b, const uint64_t* echild, uint8_t* cflag) {
  GRID_STRIDE(k, sg.E) {
    const uint8_t f = sg.ef[k];
    if (!f) continue;
    const uint64_t n = (sg.ee[k] - sg.ea[k] + b - 1) / b;
    const uint64_t c0 = echild[k];
    for (uint64_t i = 0; i < n; ++i) cflag[c0 + i] = f | (i + 1 == n ? kLastChild : 0);
  }
}

hipError_t launch_child_flags(const SegDev& sg, uint64_t b, const uint64_t* echild, uint8_t* cflag,
                              hipStream_t s) {
  if (!sg.E) return hipSuccess;
  k_child_flags<<<grid_for(sg.E, 256), 256, 0, s>>>(sg, b, echild, cflag);
  return hipGetLastError();
}

// Run of each entry, from the block its children start with.
__global__ void k_entry_runs(const uint64_t* echild, uint64_t E, const uint32_t* run,
                             uint32_t* erun) {
  GRID_STRIDE(k, E) erun[k] = run[echild[k]];
}

hipError_t launch_entry_runs(const uint64_t* echild, uint64_t E, const uint32_t* run,
                             uint32_t* erun, hipStream_t s) {
  if (!E) return hipSuccess;
  k_entry_runs<<<grid_for(E, 256), 256, 0, s>>>(echild, E, run, erun);
  return hipGetLastError();
}

// Per phase: segment k = window starts [ws[k], ws[k] + cnt - 1] (cnt into woff[k]),
// bounded by the run end sre[k]; stext[k] = the run's text.
__global__ void k_segments(PhaseArgs a, SegDev sg, uint64_t* woff) {
  GRID_STRIDE(k, sg.E) {
    const uint32_t r = sg.erun[k];
    const uint32_t t = a.lv.rtext[r];
    const uint64_t re = a.lv.re[r];
    const uint64_t L = a.Lmain;
    uint64_t Lmin = L;
    const uint64_t oL = a.odd.L[t];
    if (oL && oL < Lmin) Lmin = oL;
    const uint8_t f = sg.ef[k];
    uint64_t lo = sg.ea[k];
    if (f & kSkipInterior) {
      const uint64_t x = sg.ee[k] + 1 > L ? sg.ee[k] + 1 - L : 0;  // first start crossing e
      if (x > lo) lo = x;
    }
    uint64_t cnt = 0;
    if (a.odd.nkeys[t] && !(f & kSkipCross) && re >= Lmin) {
      uint64_t hi = sg.ee[k] - 1;
      if (re - Lmin < hi) hi = re - Lmin;
      if (hi >= lo && sg.ee[k] > lo) cnt = hi - lo + 1;
    }
    sg.ws[k] = lo;
    sg.sre[k] = re;
    sg.stext[k] = t;
    woff[k] = cnt;
  }
}

hipError_t launch_segments(const PhaseArgs& a, const SegDev& sg, uint64_t* woff, hipStream_t s) {
  if (!sg.E) return hipSuccess;
  k_segments<<<grid_for(sg.E, 256), 256, 0, s>>>(a, sg, woff);
  return hipGetLastError();
}

// Phase-2 segments from this level's phase-1 results.  A window of length b
// that starts in block Q lies inside the pair (Q, Q+1), so if that pair occurs
// earlier, so does the window: Q contributes no window starts.  Consecutive
// blocks of a run that keep their starts form one segment (their starts are
// consecutive positions).
//   k_block_seg_counts: wc[Q] = starts of Q, head[Q] = 1 where a segment begins;
//   (exclusive scans of both, totals at index c)
//   k_block_segments: segment k < S (S = head total) from its first block;
//   entries S..c repeat the window total (and name text 0), so a scan over c
//   segments works.
__global__ void k_block_seg_counts(PhaseArgs a, const uint8_t* pf, uint64_t* wc, uint64_t* head) {
  const LevelDev lv = a.lv;
  GRID_STRIDE(Q, lv.c) {
    const uint32_t t = lv.text[Q];
    const uint64_t re = lv.re[lv.run[Q]];
    const uint64_t st = lv.st[Q];
    uint64_t Lmin = a.Lmain;
    const uint64_t oL = a.odd.L[t];
    if (oL && oL < Lmin) Lmin = oL;
    uint64_t cnt = 0;
    if (a.odd.nkeys[t] && !(pf[Q] & 1) && re >= Lmin) {
      uint64_t hi = st + block_len(lv, a.tx, Q) - 1;
      if (re - Lmin < hi) hi = re - Lmin;
      if (hi >= st) cnt = hi - st + 1;
    }
    wc[Q] = cnt;
    bool h = cnt != 0;
    if (h && Q > 0 && lv.run[Q - 1] == lv.run[Q] && !(pf[Q - 1] & 1)) {
      // the previous block keeps its starts: they run up to st - 1 (a block
      // whose starts stop short of its end is the run's last with any)
      h = false;
    }
    head[Q] = h ? 1 : 0;
  }
}

__global__ void k_block_segments(PhaseArgs a, const uint64_t* wcs, const uint64_t* hs,
                                 uint64_t* ws, uint64_t* sre, uint32_t* stext, uint64_t* woff) {
  const LevelDev lv = a.lv;
  const uint64_t S = hs[lv.c], W = wcs[lv.c];
  GRID_STRIDE(k, lv.c + 1) {
    if (k < lv.c && hs[k + 1] != hs[k]) {
      const uint64_t g = hs[k];
      woff[g] = wcs[k];
      ws[g] = lv.st[k];
      sre[g] = lv.re[lv.run[k]];
      stext[g] = lv.text[k];
    }
    if (k >= S) {
      // padding: no windows, and a valid text for lanes that land here
      woff[k] = W;
      if (k < lv.c) {
        ws[k] = 0;
        sre[k] = 0;
        stext[k] = 0;
      }
    }
  }
}

hipError_t launch_block_seg_counts(const PhaseArgs& a, const uint8_t* pf, uint64_t* wc,
                                   uint64_t* head, hipStream_t s) {
  if (!a.lv.c) return hipSuccess;
  k_block_seg_counts<<<grid_for(a.lv.c, 256), 256, 0, s>>>(a, pf, wc, head);
  return hipGetLastError();
}

hipError_t launch_block_segments(const PhaseArgs& a, const uint64_t* wcs, const uint64_t* hs,
                                 uint64_t* ws, uint64_t* sre, uint32_t* stext, uint64_t* woff,
                                 hipStream_t s) {
  k_block_segments<<<grid_for(a.lv.c + 1, 256), 256, 0, s>>>(a, wcs, hs, ws, sre, stext, woff);
  return hipGetLastError();
}

// Phase-1 segments are one per entry (a parent, at most tau b window starts),
// so at the lower levels a tile of the scan would cross several of them.  An
// entry whose starts continue those of the previous entry (same run, first
// start one past the previous entry's last: adjacent parents that no fact cut
// apart) joins its segment.  Window numbers and positions stay the same; only
// the boundaries the scan has to walk go.
//   k_seg_heads: head[k] = 1 where entry k opens a merged segment (woff: the
//   scanned window counts, total at E);
//   k_seg_merge: merged segment g from the entry that opens it; entries S..E
//   repeat the window total (and name text 0), as the scan expects E of them.
__global__ void k_seg_heads(SegDev sg, const uint64_t* woff, uint64_t* head) {
  GRID_STRIDE(k, sg.E) {
    const uint64_t cnt = woff[k + 1] - woff[k];
    bool h = cnt != 0;
    if (h && k > 0) {
      const uint64_t pc = woff[k] - woff[k - 1];
      if (pc && sg.erun[k - 1] == sg.erun[k] && sg.ws[k - 1] + pc == sg.ws[k]) h = false;
    }
    head[k] = h ? 1 : 0;
  }
}

__global__ void k_seg_merge(SegDev sg, const uint64_t* woff, const uint64_t* hs, uint64_t* ws,
                            uint64_t* sre, uint32_t* stext, uint64_t* woff2) {
  const uint64_t S = hs[sg.E], W = woff[sg.E];
  GRID_STRIDE(k, sg.E + 1) {
    if (k < sg.E && hs[k + 1] != hs[k]) {
      const uint64_t g = hs[k];
      woff2[g] = woff[k];
      ws[g] = sg.ws[k];
      sre[g] = sg.sre[k];
      stext[g] = sg.stext[k];
    }
    if (k >= S) {
      woff2[k] = W;
      if (k < sg.E) {
        ws[k] = 0;
        sre[k] = 0;
        stext[k] = 0;
      }
    }
  }
}

hipError_t launch_seg_heads(const SegDev& sg, const uint64_t* woff, uint64_t* head, hipStream_t s) {
  if (!sg.E) return hipSuccess;
  k_seg_heads<<<grid_for(sg.E, 256), 256, 0, s>>>(sg, woff, head);
  return hipGetLastError();
}

hipError_t launch_seg_merge(const SegDev& sg, const uint64_t* woff, const uint64_t* hs, uint64_t* ws,
                            uint64_t* sre, uint32_t* stext, uint64_t* woff2, hipStream_t s) {
  k_seg_merge<<<grid_for(sg.E + 1, 256), 256, 0, s>>>(sg, woff, hs, ws, sre, stext, woff2);
  return hipGetLastError();
}

// ---------------------------------------------------------------- probe scan (a4, a6)

constexpr int kScanK = 16;                      // windows per lane per chunk
constexpr int kScanSlowGroup = 4;                // steps whose loads leave together where a chunk crosses segments
constexpr uint64_t kScanChunk = 64ull * kScanK;  // windows per wave per chunk
static_assert(kScanChunk == kProbeTile, "the host counts algorithmic bytes per tile of kProbeTile windows");
static_assert(kLeanK == kScanK, "lean scans take the same chunks");

// Windows are numbered run after run (woff = exclusive prefix of per-run window
// counts).  Each wave takes chunks of 64*kScanK consecutive window numbers;
// in step k lane l handles window chunk + 64k + l, so consecutive lanes read
// consecutive prefix fingerprints.
//
// Before touching the table, a window's hash is tested against a bit filter of
// the phase's keys (one or two bits per key, set by k_keys) that every
// workgroup first copies into LDS.  A clear bit proves that no key has this
// hash.  The windows that pass are appended to a per-wave queue in LDS (ballot
// + prefix popcount) and probed 64 at a time.
constexpr int kProbeThreads = 1024;

__device__ __forceinline__ bool filter_has(const uint32_t* s_filt, uint64_t b1, uint64_t b2) {
  return ((s_filt[b1 >> 5] >> (b1 & 31)) & (s_filt[b2 >> 5] >> (b2 & 31)) & 1) != 0;
}


// MODE 0 (kept in the template, not launched): no filter, every window probes
// the table.  MODE 1: filter, and the
// windows that pass go to a per-wave LDS queue; 64 queued windows at a time
// then form their fingerprints and probe together, so a wave waits for one
// round of loads per 64 candidates rather than per step.  MODE 2: filter,
// candidates probe at once (no queue; texts beyond the queue's packing).
//
// PRE (MODE 1 only): the filter holds bits of the keys' 32-bit hashes
// (H[i+L] - H[i] x32^L mod 2^32), and the scan reads only H for every window;
// the 61-bit fingerprint is formed for queued windows alone.  Equal strings
// have equal hashes of both kinds, so every occurrence of a key still reaches
// the table; a window that agrees with a key in both hashes without being an
// occurrence is a collision, caught by the same verification as before.
//
// A chunk in which every lane's 16 windows lie inside that lane's current
// segment (the usual case on long runs) takes a straight-line path that issues
// eight windows' hash loads together, before using any of them.
//
// LEAN: the 32-bit hashes are sampled (memory-lean builds) and lanes roll them
// along consecutive windows (lean.hpp).  Queued windows form their 61-bit
// fingerprints from dense prefix fingerprints when the build keeps them, else
// from the samples.
//
// Instances without a short final key hold their registers (SGPRs included)
// to two 1024-thread workgroups per CU, 8 waves per SIMD.  Instances with one
// carry more live values (and load the short key's hashes with the main ones):
// they run one workgroup per CU with up to 128 VGPRs, which measured faster
// than spilling at 64.
template <int MODE, bool ODD, bool SALT, bool PRE, bool LEAN>
__global__ __launch_bounds__(kProbeThreads) __attribute__((amdgpu_waves_per_eu(ODD ? 4 : 8)))
void k_probe_scan(PhaseArgs a, const uint64_t* __restrict__ woff) {
  constexpr bool FILTER = MODE != 0;
  static_assert(!PRE || MODE == 1, "the 32-bit hash feeds the queued filter only");
  static_assert(!LEAN || MODE == 1, "sampled prefixes serve queued candidates only");
  extern __shared__ uint64_t s_lds[];
  const uint32_t fbits = a.filt_bits;
  const bool two = a.filt_two != 0;
  uint32_t* s_filt = reinterpret_cast<uint32_t*>(s_lds);
  if (FILTER) {
    const uint32_t nq = (uint32_t)(1ull << (fbits - 7));  // uint4 words
    const uint4* src = reinterpret_cast<const uint4*>(a.filt);
    uint4* dst = reinterpret_cast<uint4*>(s_filt);
    for (uint32_t q = threadIdx.x; q < nq; q += blockDim.x) dst[q] = src[q];
    __syncthreads();
  }
  const int lane = lane_id();
  uint64_t* q = s_lds + (FILTER ? (1ull << (fbits - 6)) : 0) + (uint64_t)(threadIdx.x >> 6) * kQueue;
  uint32_t qn = 0;  // wave-uniform queue length

  const uint64_t R = a.lv.R;
  const uint64_t W = woff[R];
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t* __restrict__ P = a.P;
  const uint32_t* __restrict__ H = a.P32;
  const uint64_t* __restrict__ rs_ = a.lv.rs;
  const uint64_t* __restrict__ re_ = a.lv.re;
  const uint64_t L = a.Lmain, xL = a.xLmain, fmask = a.fpmask;
  const uint32_t x32L = a.x32L;
  Slot* __restrict__ slots = a.tab.slots;
  const uint64_t mask = a.tab.mask;

  const auto fp61 = [&](uint64_t i, uint64_t salt) {
    uint64_t f = P ? sub61(P[i + L], mul61(P[i], xL)) : win61<true>(a, i, L, xL);
    if (SALT) f = add61(f, salt);
    return f & fmask;
  };
  const auto pass32 = [&](uint32_t h) {
    const uint32_t b1 = filter_bit32(h, fbits);
    return filter_has(s_filt, b1, two ? filter_bit32b(h, fbits) : b1);
  };
  const uint64_t* __restrict__ filt2 = reinterpret_cast<const uint64_t*>(a.filt2);
  const uint32_t f2words = a.filt2_words;
  const auto pass2 = [&](uint32_t h) {
    const uint64_t m = filter2_mask(h);
    return (filt2[filter2_word(h, f2words)] & m) == m;
  };
  const auto pass61 = [&](uint64_t f) {
    const uint64_t b1 = filter_bit(f, fbits);
    return filter_has(s_filt, b1, two ? filter_bit2(f, fbits) : b1);
  };
  // the entry this lane holds: form its fingerprint and probe
  const auto probe_entry = [&](uint64_t e) {
    const uint64_t i = e & kQPosMask;
    const uint64_t salt = SALT ? a.tx.tsalt[e >> kQPosBits] : 0;
    probe(slots, mask, fp61(i, salt), i);
  };
  // whole wave: append the lanes' candidates; probe 64 once 64 are waiting
  uint64_t ncand = 0;  // wave-uniform: windows that passed the filters
  const auto push = [&](bool cand, uint64_t i, uint32_t t) {
    const uint64_t bal = __ballot(cand);
    if (!bal) return;
    const uint32_t my = (uint32_t)__popcll(bal & ((1ull << lane) - 1));
    if (cand) q[qn + my] = ((uint64_t)t << kQPosBits) | i;
    qn += (uint32_t)__popcll(bal);
    ncand += (uint64_t)__popcll(bal);
    if (qn >= 64) {
      wave_sync();
      const uint64_t e = q[lane];
      const bool mv = (uint32_t)lane < qn - 64;
      const uint64_t e2 = mv ? q[64 + lane] : 0;
      wave_sync();
      if (mv) q[lane] = e2;
      qn -= 64;
      probe_entry(e);
      wave_sync();
    }
  };

  for (uint64_t ch = gw; ch * kScanChunk < W; ch += nw) {
    if constexpr (LEAN) {
      // sampled hashes: consecutive windows per lane, rolled (lean.hpp)
      const auto test8 = [&](const uint32_t* hv, bool* ok) {
#pragma unroll
        for (int k = 0; k < 8; ++k) ok[k] = pass32(hv[k]);
        if (f2words) {
          uint64_t wv[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) wv[k] = ok[k] ? filt2[filter2_word(hv[k], f2words)] : ~0ull;
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const uint64_t m = filter2_mask(hv[k]);
            ok[k] = ok[k] && (wv[k] & m) == m;
          }
        }
      };
      const auto test1 = [&](uint32_t h) { return pass32(h) && (!f2words || pass2(h)); };
      lean_chunk<ODD, ODD || SALT, SALT>(a, woff, 0, R, W, ch * kScanChunk + (uint64_t)lane * kLeanK,
                                         [](uint32_t) {}, test8, test1, push);
      continue;
    }
    const uint64_t w0 = ch * kScanChunk + lane;
    uint64_t lo = 0, hi = R;
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (woff[mid] <= w0) lo = mid; else hi = mid;
    }
    uint64_t r = lo;
    uint64_t wo = woff[r], wn = woff[r + 1], rs = rs_[r], re = re_[r];
    // lanes past the last window hold no segment: they read no text entry
    uint32_t t = ((ODD || SALT) && w0 < W) ? a.lv.rtext[r] : 0;
    uint64_t salt = SALT ? a.tx.tsalt[t] : 0;
    // the text's short final key, if any (kept in registers while t holds)
    uint64_t oL = 0, opos = 0;
    uint32_t oh = 0, ox = 0;
    const auto load_odd = [&]() {
      oL = a.odd.L[t];
      if (oL) {
        opos = a.odd.pos[t];
        const uint64_t hx = a.odd.h32[t];
        oh = (uint32_t)hx;
        ox = (uint32_t)(hx >> 32);
      }
    };
    if (ODD && w0 < W) load_odd();
    // the short key's 61-bit fingerprint at i, against the key's (text t)
    const auto odd61 = [&](uint64_t i, uint64_t sl) {
      uint64_t g = P ? sub61(P[i + oL], mul61(P[i], a.odd.xp[t])) : win61<true>(a, i, oL, a.odd.xp[t]);
      if (SALT) g = add61(g, sl);
      if ((g & fmask) == a.odd.fp[t] && i < a.odd.best[t])
        atomicMin((unsigned long long*)&a.odd.best[t], (unsigned long long)i);
    };

    // (the short final key's windows, shorter than the main ones, fit wherever
    // a main window does; the unqueued scan tests it on the per-step path)
    if (!ODD || PRE) {
      const uint64_t wl = w0 + 64ull * (kScanK - 1);
      const bool lane_ok = wl < wn && rs + (wl - wo) + L <= re;
      if (__ballot(lane_ok) == ~0ull) {
        const uint64_t i0 = rs + (w0 - wo);
#pragma unroll
        for (int k0 = 0; k0 < kScanK; k0 += 8) {
          if (PRE) {
            const uint32_t s32 = SALT ? (uint32_t)salt : 0u;
            // the sixteen loads leave together: the scheduler would otherwise
            // pair each load with its use and wait out every latency in turn
            uint32_t ha[8], hb[8], hc[8];
            // (and the short key's, H[i + oL], where the text has one)
            const bool oddk = ODD && oL;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const uint64_t i = i0 + 64ull * (k0 + k);
              hb[k] = H[i + L];
              ha[k] = H[i];
              if (oddk) hc[k] = H[i + oL];
            }
            __builtin_amdgcn_sched_barrier(0);
            uint32_t hv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) hv[k] = hb[k] - ha[k] * x32L + s32;
            if (oddk) {
              // the short key's 32-bit hashes (loaded with the others); the rare
              // matches form their 61-bit fingerprints one at a time
              uint32_t om = 0;
#pragma unroll
              for (int k = 0; k < 8; ++k) {
                const uint64_t i = i0 + 64ull * (k0 + k);
                if (i < opos && hc[k] - ha[k] * ox + s32 == oh) om |= 1u << k;
              }
              while (om) {
                const int k = __builtin_ctz(om);
                om &= om - 1;
                odd61(i0 + 64ull * (k0 + k), salt);
              }
            }
            bool ok[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) ok[k] = pass32(hv[k]);
            if (f2words) {
              // second filter: the eight steps' loads are issued together
              uint64_t wv[8];
#pragma unroll
              for (int k = 0; k < 8; ++k) wv[k] = ok[k] ? filt2[filter2_word(hv[k], f2words)] : ~0ull;
#pragma unroll
              for (int k = 0; k < 8; ++k) {
                const uint64_t m = filter2_mask(hv[k]);
                ok[k] = ok[k] && (wv[k] & m) == m;
              }
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) push(ok[k], i0 + 64ull * (k0 + k), t);
          } else {
            uint64_t fv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) fv[k] = fp61(i0 + 64ull * (k0 + k), salt);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const uint64_t i = i0 + 64ull * (k0 + k);
              const bool cand = FILTER ? pass61(fv[k]) : true;
              if (MODE == 1) {
                push(cand, i, t);
              } else {
                ncand += (uint64_t)__popcll(__ballot(cand));
                if (cand) probe(slots, mask, fv[k], i);
              }
            }
          }
        }
        continue;
      }
    }

    if constexpr (PRE && !SALT) {
      // One text (its short key stays): the chunk crosses segments.  Per group
      // of steps each lane first follows its windows across the segments, then
      // the group's loads leave together.
#pragma unroll
      for (int k0 = 0; k0 < kScanK; k0 += kScanSlowGroup) {
        uint64_t ik[kScanSlowGroup];
        uint32_t vm = 0, om = 0;  // steps with a main-length window, with a short-key window
#pragma unroll
        for (int k = 0; k < kScanSlowGroup; ++k) {
          const uint64_t w = w0 + 64ull * (k0 + k);
          const bool live = w < W;
          if (live && w >= wn) {
            do {
              ++r;
              wo = wn;
              wn = woff[r + 1];
            } while (w >= wn);
            rs = rs_[r];
            re = re_[r];
          }
          const uint64_t i = rs + (w - wo);
          ik[k] = i;
          if (live && i + L <= re) vm |= 1u << k;
          if (ODD && live && oL && i + oL <= re && i < opos) om |= 1u << k;
        }
        uint32_t ha[kScanSlowGroup], hb[kScanSlowGroup], hc[kScanSlowGroup];
#pragma unroll
        for (int k = 0; k < kScanSlowGroup; ++k) {
          hb[k] = ((vm >> k) & 1) ? H[ik[k] + L] : 0u;
          ha[k] = (((vm | om) >> k) & 1) ? H[ik[k]] : 0u;
          if (ODD) hc[k] = ((om >> k) & 1) ? H[ik[k] + oL] : 0u;
        }
        __builtin_amdgcn_sched_barrier(0);
        if (ODD) {
          uint32_t mm = 0;
#pragma unroll
          for (int k = 0; k < kScanSlowGroup; ++k)
            if (((om >> k) & 1) && hc[k] - ha[k] * ox == oh) mm |= 1u << k;
          while (mm) {
            const int k = __builtin_ctz(mm);
            mm &= mm - 1;
            odd61(ik[k], 0);
          }
        }
        uint32_t hv[kScanSlowGroup];
        bool ok[kScanSlowGroup];
#pragma unroll
        for (int k = 0; k < kScanSlowGroup; ++k) {
          hv[k] = hb[k] - ha[k] * x32L;
          ok[k] = ((vm >> k) & 1) && pass32(hv[k]);
        }
        if (f2words) {
          uint64_t wv[kScanSlowGroup];
#pragma unroll
          for (int k = 0; k < kScanSlowGroup; ++k) wv[k] = ok[k] ? filt2[filter2_word(hv[k], f2words)] : ~0ull;
#pragma unroll
          for (int k = 0; k < kScanSlowGroup; ++k) {
            const uint64_t m = filter2_mask(hv[k]);
            ok[k] = ok[k] && (wv[k] & m) == m;
          }
        }
#pragma unroll
        for (int k = 0; k < kScanSlowGroup; ++k) push(ok[k], ik[k], t);
      }
      continue;
    }

    for (int k = 0; k < kScanK; ++k) {
      const uint64_t w = w0 + (uint64_t)k * 64;
      const bool live = w < W;  // every lane stays in the loop (the queue is wave-wide)
      if (live && w >= wn) {
        do {
          ++r;
          wo = wn;
          wn = woff[r + 1];
        } while (w >= wn);
        rs = rs_[r];
        re = re_[r];
        if (ODD || SALT) t = a.lv.rtext[r];
        if (SALT) salt = a.tx.tsalt[t];
        if (ODD) load_odd();
      }
      const uint64_t i = rs + (w - wo);
      bool cand = false;
      if (live && i + L <= re) {
        if (PRE) {
          const uint32_t h = H[i + L] - H[i] * x32L + (SALT ? (uint32_t)salt : 0u);
          cand = pass32(h) && (!f2words || pass2(h));
        } else {
          const uint64_t f = fp61(i, salt);
          cand = FILTER ? pass61(f) : true;
          if (MODE != 1 && cand) probe(slots, mask, f, i);
        }
      }
      if (MODE == 1) push(cand, i, t);
      else ncand += (uint64_t)__popcll(__ballot(cand));
      // the short key: its 32-bit hash first (equal strings always agree),
      // the 61-bit fingerprint only where that matches
      if (ODD && live && oL && i + oL <= re && i < opos) {
        const uint32_t ho = H[i + oL] - H[i] * ox + (SALT ? (uint32_t)salt : 0u);
        if (ho == oh) odd61(i, salt);
      }
    }
  }
  if (MODE == 1 && qn) {
    wave_sync();
    if ((uint32_t)lane < qn) probe_entry(q[lane]);
  }
  if (a.pc && lane == 0 && ncand) atomicAdd((unsigned long long*)(a.pc + kPcCand), (unsigned long long)ncand);
}

// Dynamic LDS beyond 64 KiB has to be allowed per kernel.
static hipError_t allow_lds(const void* fn, size_t bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_probe_scan(const PhaseArgs& a, const uint64_t* woff, bool has_odd,
                             bool has_salt, uint64_t max_windows, int mode, hipStream_t s) {
  if (a.lv.R == 0) return hipSuccess;
  const uint64_t waves = (max_windows + kScanChunk - 1) / kScanChunk;
  // two 1024-thread workgroups per CU: LDS of at most 80 KiB each (mode 1:
  // filter up to 64 KiB + queues 16 KiB; mode 2: filter up to 64 KiB)
  const unsigned grid = grid_for(waves * 64, kProbeThreads, 512);
  size_t lds = 0;
  if (mode == 1)
    lds = ((size_t)1 << (a.filt_bits - 3)) + (size_t)(kProbeThreads / 64) * kQueue * 8;
  else if (mode == 2)
    lds = (size_t)1 << (a.filt_bits - 3);
  // the keys filled the filter from the hash kind that pre32 names
  if (a.pre32 && mode != 1) return hipErrorInvalidValue;
  const bool pre = a.pre32 != 0;
#define BT_PROBE_LAUNCH(M, O, S, Q, LN)                                                  \
  do {                                                                                   \
    if (lds > 65536) {                                                                   \
      const hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_probe_scan<M, O, S, Q, LN>), lds); \
      if (e != hipSuccess) return e;                                                     \
    }                                                                                    \
    k_probe_scan<M, O, S, Q, LN><<<grid, kProbeThreads, lds, s>>>(a, woff);              \
  } while (0)
#define BT_PROBE_SALT(M, O, Q, LN) \
  if (has_salt) BT_PROBE_LAUNCH(M, O, true, Q, LN); else BT_PROBE_LAUNCH(M, O, false, Q, LN);
  // sampled fingerprints serve queued candidates only; sampled 32-bit hashes
  // take the rolled window loop (the LEAN instances)
  if (a.P == nullptr && mode != 1) return hipErrorInvalidValue;
  const bool lean = a.P32 == nullptr;
  if (mode == 1) {
    if (!pre) return hipErrorInvalidValue;  // queued scans always pre-filter
    if (lean) {
      if (has_odd) {
        BT_PROBE_SALT(1, true, true, true)
      } else {
        BT_PROBE_SALT(1, false, true, true)
      }
    } else if (has_odd) {
      BT_PROBE_SALT(1, true, true, false)
    } else {
      BT_PROBE_SALT(1, false, true, false)
    }
  } else if (mode == 2) {
    if (has_odd) {
      BT_PROBE_SALT(2, true, false, false)
    } else {
      BT_PROBE_SALT(2, false, false, false)
    }
  } else {
    return hipErrorInvalidValue;  // every scan filters (mode 1 or 2)
  }
#undef BT_PROBE_SALT
#undef BT_PROBE_LAUNCH
  return hipGetLastError();
}

// ---------------------------------------------------------------- byte scan (a4)
//
// For phases with few keys (the upper levels, whose blocks are longer than the
// spacing of the text's differences, so that no window is skipped), reading
// two prefix hashes per window is the whole cost.  Here a window is first
// tested on its own first eight bytes against a filter of the keys' first
// eight bytes: 1 byte of text per window instead of 8 bytes of hashes.  Equal
// strings share their first eight bytes, so every occurrence of a key passes.
// The windows that pass (in a repetitive text, mostly true copies of a key's
// first eight bytes) go to the per-wave LDS queue of the probe scan and form
// their 61-bit fingerprints 64 at a time.
//
// A wave takes 1024 consecutive window numbers; lane l takes 16 consecutive
// ones.  When they lie in one segment the lane loads the 28 aligned bytes that
// cover them and takes each window's eight bytes with byte-aligns.
constexpr int kByteThreads = 1024;
constexpr int kByteK = 16;  // windows per lane
// Queue entries: position in bits 0..39, text in bits 40..62, and bit 63 set
// when the main-length window does not fit its run.
constexpr uint64_t kByteTextMask = (1ull << 23) - 1;

template <bool ODD, bool SALT, bool LEAN>
__global__ __launch_bounds__(kByteThreads) __attribute__((amdgpu_waves_per_eu(8)))
void k_byte_scan(PhaseArgs a, const uint64_t* __restrict__ woff) {
  extern __shared__ uint64_t s_lds[];
  uint32_t* s_bf = reinterpret_cast<uint32_t*>(s_lds);
  const uint32_t bits = a.bfilt_bits;
  {
    const uint32_t nq = 1u << (bits - 7);  // uint4 words
    const uint4* src = reinterpret_cast<const uint4*>(a.bfilt);
    uint4* dst = reinterpret_cast<uint4*>(s_bf);
    for (uint32_t k = threadIdx.x; k < nq; k += blockDim.x) dst[k] = src[k];
    __syncthreads();
  }
  const int lane = lane_id();
  uint64_t* q = s_lds + (1ull << (bits - 6)) + (uint64_t)(threadIdx.x >> 6) * kQueue;
  uint32_t qn = 0;  // wave-uniform queue length
  const uint64_t R = a.lv.R;
  const uint64_t W = woff[R];
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint8_t* __restrict__ T = a.T;
  const uint64_t* __restrict__ P = a.P;
  const uint64_t L = a.Lmain, xL = a.xLmain, fmask = a.fpmask;
  Slot* __restrict__ slots = a.tab.slots;
  const uint64_t mask = a.tab.mask;
  const auto has = [&](uint32_t lo, uint32_t hi) {
    const uint32_t b = prefix8_bit(lo, hi, bits);
    return ((s_bf[b >> 5] >> (b & 31)) & 1u) != 0;
  };
  // A queued window: its fingerprints against the keys.  Bit 63 of the entry
  // says whether the main-length window fits its run.  A window of the short
  // final key's length always fits (segments hold the windows of the shorter
  // of the two lengths), so only the text's end bounds it.
  const auto check = [&](uint64_t e) {
    const uint64_t i = e & kQPosMask;
    const uint32_t t = (uint32_t)((e >> kQPosBits) & kByteTextMask);  // bit 63 is the fit bit
    const uint64_t salt = SALT ? a.tx.tsalt[t] : 0;
    if (!(e >> 63)) {
      uint64_t f = P ? sub61(P[i + L], mul61(P[i], xL)) : win61<true>(a, i, L, xL);
      if (SALT) f = add61(f, salt);
      probe(slots, mask, f & fmask, i);
    }
    if (ODD) {
      const uint64_t oL = a.odd.L[t];
      if (oL && i + oL <= a.tx.tend[t] && i < a.odd.pos[t]) {
        uint64_t g = P ? sub61(P[i + oL], mul61(P[i], a.odd.xp[t])) : win61<true>(a, i, oL, a.odd.xp[t]);
        if (SALT) g = add61(g, salt);
        if ((g & fmask) == a.odd.fp[t] && i < a.odd.best[t])
          atomicMin((unsigned long long*)&a.odd.best[t], (unsigned long long)i);
      }
    }
  };
  // whole wave: append the lanes' candidates; check 64 once 64 are waiting.
  // Bit 63 of an entry: the main-length window does not fit the run.
  uint64_t ncand = 0;  // wave-uniform: windows that passed the filter
  const auto push = [&](bool cand, uint64_t e) {
    const uint64_t bal = __ballot(cand);
    if (!bal) return;
    const uint32_t my = (uint32_t)__popcll(bal & ((1ull << lane) - 1));
    if (cand) q[qn + my] = e;
    qn += (uint32_t)__popcll(bal);
    ncand += (uint64_t)__popcll(bal);
    if (qn >= 64) {
      wave_sync();
      const uint64_t e0 = q[lane];
      const bool mv = (uint32_t)lane < qn - 64;
      const uint64_t e2 = mv ? q[64 + lane] : 0;
      wave_sync();
      if (mv) q[lane] = e2;
      qn -= 64;
      check(e0);
      wave_sync();
    }
  };

  for (uint64_t ch = gw; ch * (64ull * kByteK) < W; ch += nw) {
    const uint64_t w0 = ch * (64ull * kByteK) + (uint64_t)lane * kByteK;
    const bool any = w0 < W;  // lanes past the last window hold no segment
    uint64_t r = 0, wo = 0, wn = 0, rs = 0, re = 0;
    uint32_t t = 0;
    if (any) {
      uint64_t lo = 0, hi = R;
      while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) >> 1;
        if (woff[mid] <= w0) lo = mid; else hi = mid;
      }
      r = lo;
      wo = woff[r];
      wn = woff[r + 1];
      rs = a.lv.rs[r];
      re = a.lv.re[r];
      t = a.lv.rtext[r];
    }
    const uint64_t i0 = rs + (w0 - wo);
    // the lane's 16 windows in one segment, all of main length inside the run
    const bool fast = any && w0 + (kByteK - 1) < wn && i0 + (kByteK - 1) + L <= re;
    uint32_t m = 0;  // bit k: window w0 + k passes
    if (fast) {
      // The 28 bytes from the 4-byte aligned address at or below T + i0 cover
      // [i0, i0 + 23).  They end inside the lane's last window, which ends at
      // or before the run end (L >= 16 > 12: keys of the byte scan are blocks
      // or pairs of blocks of b >= 16), and they start no lower than the
      // aligned base of the allocation holding the text.
      const uintptr_t ad = reinterpret_cast<uintptr_t>(T + i0);
      const uint32_t* wp = reinterpret_cast<const uint32_t*>(ad & ~(uintptr_t)3);
      uint32_t w[7];
#pragma unroll
      for (int k = 0; k < 7; ++k) w[k] = wp[k];
      const uint32_t sh = (uint32_t)(ad & 3);
      uint32_t x[6];  // x[k] = bytes [i0 + 4k, i0 + 4k + 4)
#pragma unroll
      for (int k = 0; k < 6; ++k) x[k] = __builtin_amdgcn_alignbyte(w[k + 1], w[k], sh);
#pragma unroll
      for (int k = 0; k < kByteK; ++k) {
        const int qq = k >> 2, o = k & 3;
        const uint32_t l4 = o ? __builtin_amdgcn_alignbyte(x[qq + 1], x[qq], o) : x[qq];
        const uint32_t h4 = o ? __builtin_amdgcn_alignbyte(x[qq + 2], x[qq + 1], o) : x[qq + 1];
        m |= (has(l4, h4) ? 1u : 0u) << k;
      }
    } else if (any) {
      // windows across segment ends: walk them one by one (this lane only)
      uint64_t r2 = r, wo2 = wo, wn2 = wn, rs2 = rs;
      for (int k = 0; k < kByteK; ++k) {
        const uint64_t wi = w0 + k;
        if (wi >= W) break;
        while (wi >= wn2) {
          ++r2;
          wo2 = wn2;
          wn2 = woff[r2 + 1];
          rs2 = a.lv.rs[r2];
        }
        // every window of a segment has at least 8 bytes before the run end
        const uint64_t i = rs2 + (wi - wo2);
        uint32_t l4 = 0, h4 = 0;
        for (int b = 0; b < 4; ++b) {
          l4 |= (uint32_t)T[i + b] << (8 * b);
          h4 |= (uint32_t)T[i + 4 + b] << (8 * b);
        }
        m |= (has(l4, h4) ? 1u : 0u) << k;
      }
    }
    if (!__ballot(m != 0)) continue;  // most chunks hold no candidate
    // queue the candidates, 16 wave-wide steps; lanes that walked segments
    // walk them again, now with the run end and text of each window
    for (int k = 0; k < kByteK; ++k) {
      uint64_t e = 0;
      const bool c = (m >> k) & 1u;
      if (c) {
        const uint64_t wi = w0 + k;
        if (!fast) {
          while (wi >= wn) {
            ++r;
            wo = wn;
            wn = woff[r + 1];
            rs = a.lv.rs[r];
            re = a.lv.re[r];
            t = a.lv.rtext[r];
          }
        }
        const uint64_t i = rs + (wi - wo);
        e = ((i + L > re) ? (1ull << 63) : 0) | ((uint64_t)t << kQPosBits) | i;
      }
      push(c, e);
    }
  }
  if (qn) {
    wave_sync();
    if ((uint32_t)lane < qn) check(q[lane]);
  }
  if (a.pc && lane == 0 && ncand) atomicAdd((unsigned long long*)(a.pc + kPcCand), (unsigned long long)ncand);
}

hipError_t launch_byte_scan(const PhaseArgs& a, const uint64_t* woff, bool has_odd, bool has_salt,
                            uint64_t max_windows, hipStream_t s) {
  if (a.lv.R == 0) return hipSuccess;
  if (a.bfilt_bits < 12 || a.bfilt_bits > 19) return hipErrorInvalidValue;
  const uint64_t waves = (max_windows + 64 * kByteK - 1) / (64 * kByteK);
  const unsigned grid = grid_for(waves * 64, kByteThreads, 512);
  // filter up to 64 KiB + queues 16 KiB: two 1024-thread workgroups per CU
  const size_t lds = ((size_t)1 << (a.bfilt_bits - 3)) + (size_t)(kByteThreads / 64) * kQueue * 8;
#define BT_BYTE_LAUNCH(O, S, LN)                                                           \
  do {                                                                                     \
    if (lds > 65536) {                                                                     \
      const hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_byte_scan<O, S, LN>), lds); \
      if (e != hipSuccess) return e;                                                       \
    }                                                                                      \
    k_byte_scan<O, S, LN><<<grid, kByteThreads, lds, s>>>(a, woff);                        \
  } while (0)
#define BT_BYTE_SALT(O, LN) \
  if (has_salt) BT_BYTE_LAUNCH(O, true, LN); else BT_BYTE_LAUNCH(O, false, LN);
  if (a.P == nullptr) {
    if (has_odd) {
      BT_BYTE_SALT(true, true)
    } else {
      BT_BYTE_SALT(false, true)
    }
  } else if (has_odd) {
    BT_BYTE_SALT(true, false)
  } else {
    BT_BYTE_SALT(false, false)
  }
#undef BT_BYTE_SALT
#undef BT_BYTE_LAUNCH
  return hipGetLastError();
}

// ---------------------------------------------------------------- resolve / verify / retry

// Keys whose slot minimum is their own position are their own leftmost
// occurrence; the rest are appended to the verification list.  Returning
// atomics on one address serialize (about 10 ns apart), so a 1024-thread
// workgroup claims its whole share of the list with a single update.
constexpr int kResolveThreads = 1024;

__global__ __launch_bounds__(kResolveThreads) void k_resolve(PhaseArgs a, VerifyBufs v) {
  __shared__ uint32_t s_w[kResolveThreads / 64];
  __shared__ unsigned long long s_base;
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  const uint64_t c = a.lv.c;
  for (uint64_t j0 = (uint64_t)blockIdx.x * kResolveThreads; j0 < c;
       j0 += (uint64_t)gridDim.x * kResolveThreads) {
    const uint64_t j = j0 + threadIdx.x;
    bool need = false;
    uint64_t best = 0;
    if (j < c) {
      const uint32_t s = a.k.slot[j];
      if (s != kNoKey && s != kCopyKey) {
        const uint64_t pos = a.lv.st[j];
        best = (s == kOddKey) ? a.odd.best[a.lv.text[j]] : a.tab.slots[s].best;
        if (best == pos) a.k.lm[j] = pos;
        else need = true;
      }
    }
    const uint64_t bal = __ballot(need);
    if (lane == 0) s_w[wv] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t tot = 0;
      for (int q = 0; q < kResolveThreads / 64; ++q) {
        const uint32_t n = s_w[q];
        s_w[q] = tot;
        tot += n;
      }
      s_base = tot ? atomicAdd((unsigned long long*)&v.counts[0], (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    if (need) {
      const uint64_t idx = s_base + s_w[wv] + __popcll(bal & ((1ull << lane) - 1));
      v.vlist[idx] = (uint32_t)j;
      v.vbest[idx] = best;
      v.vmis[idx] = 0;
    }
    __syncthreads();  // s_w and s_base are reused
  }
}

hipError_t launch_resolve(const PhaseArgs& a, const VerifyBufs& v, hipStream_t s) {
  k_resolve<<<grid_for(a.lv.c, kResolveThreads, 2048), kResolveThreads, 0, s>>>(a, v);
  return hipGetLastError();
}

__global__ void k_phase_record(uint64_t* pc, const uint64_t* windows, const uint64_t* counts) {
  if (threadIdx.x == 0) {
    pc[kPcWindows] = windows ? *windows : 0;
    pc[kPcVerified] = counts[0];
    pc[kPcCollisions] = counts[1];
  }
}

hipError_t launch_phase_record(uint64_t* pc, const uint64_t* windows, const VerifyBufs& v,
                               hipStream_t s) {
  k_phase_record<<<1, 64, 0, s>>>(pc, windows, v.counts);
  return hipGetLastError();
}

constexpr uint64_t kVChunk = 4096;  // bytes compared per work item

// One wave compares up to 4 KiB of a key with the candidate occurrence.
__device__ __forceinline__ bool wave_bytes_differ(const uint8_t* __restrict__ T, uint64_t a0,
                                                  uint64_t b0, uint64_t off, uint64_t end) {
  bool diff = false;
  for (uint64_t o = off + (uint64_t)lane_id() * 16; o < end; o += 64 * 16) {
    if (o + 16 <= end) {
      const uint4 x = load16(T + a0 + o);
      const uint4 y = load16(T + b0 + o);
      diff |= (x.x != y.x) | (x.y != y.y) | (x.z != y.z) | (x.w != y.w);
    } else {
      for (uint64_t q = o; q < end; ++q) diff |= T[a0 + q] != T[b0 + q];
    }
  }
  return __any(diff);
}

// Items are (key, 4 KiB chunk) pairs.  A group of G lanes (G = 64 for keys of
// 1 KiB or more, fewer for short keys so that several keys share a wave)
// compares one item, 16 bytes per lane per step.
template <int G>
__global__ __launch_bounds__(256) void k_verify(PhaseArgs a, VerifyBufs v, uint64_t cpk) {
  const uint64_t cnt = v.counts[0];
  const uint64_t items = cnt * cpk;
  const int lane = lane_id();
  const int sub = lane % G;
  const uint64_t ggrp = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const uint64_t ngrp = ((uint64_t)gridDim.x * blockDim.x) / G;
  // every lane of a wave runs the same number of iterations (the group
  // reduction below is a wave-wide ballot)
  const uint64_t iters = (items + ngrp - 1) / ngrp;
  for (uint64_t k = 0; k < iters; ++k) {
    const uint64_t it = ggrp + k * ngrp;
    bool diff = false;
    bool mine = false;
    uint64_t idx = 0;
    if (it < items) {
      idx = it / cpk;
      const uint64_t chunk = it - idx * cpk;
      const uint32_t j = v.vlist[idx];
      const uint64_t best = v.vbest[idx];
      const uint64_t pos = a.lv.st[j];
      const uint64_t L = a.k.len[j];
      if (best < a.tx.tstart[a.lv.text[j]]) {  // hit in another text: a collision
        diff = true;
        mine = true;
      } else {
        const uint64_t off = chunk * kVChunk;
        if (off < L) {
          mine = true;
          const uint64_t end = L - off < kVChunk ? L : off + kVChunk;
          for (uint64_t o = off + (uint64_t)sub * 16; o < end; o += (uint64_t)G * 16) {
            if (o + 16 <= end) {
              const uint4 x = load16(a.T + best + o);
              const uint4 y = load16(a.T + pos + o);
              diff |= (x.x != y.x) | (x.y != y.y) | (x.z != y.z) | (x.w != y.w);
            } else {
              for (uint64_t q = o; q < end; ++q) diff |= a.T[best + q] != a.T[pos + q];
            }
          }
        }
      }
    }
    const uint64_t bal = __ballot(diff);
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1) << (lane - sub));
    if (mine && sub == 0 && (bal & gmask)) v.vmis[idx] = 1;
  }
}

hipError_t launch_verify(const PhaseArgs& a, const VerifyBufs& v, uint64_t max_len,
                         hipStream_t s) {
  const uint64_t cpk = max_len ? (max_len + kVChunk - 1) / kVChunk : 1;
  const uint64_t items = a.lv.c * cpk;
  // lanes per item: about one 16-byte word per lane, at least 4 lanes
  if (max_len <= 64) {
    k_verify<4><<<grid_for(items * 4, 256, 2048), 256, 0, s>>>(a, v, cpk);
  } else if (max_len <= 128) {
    k_verify<8><<<grid_for(items * 8, 256, 2048), 256, 0, s>>>(a, v, cpk);
  } else if (max_len <= 256) {
    k_verify<16><<<grid_for(items * 16, 256, 2048), 256, 0, s>>>(a, v, cpk);
  } else if (max_len <= 512) {
    k_verify<32><<<grid_for(items * 32, 256, 2048), 256, 0, s>>>(a, v, cpk);
  } else {
    k_verify<64><<<grid_for(items * 64, 256, 2048), 256, 0, s>>>(a, v, cpk);
  }
  return hipGetLastError();
}

__global__ void k_finish(PhaseArgs a, VerifyBufs v) {
  const uint64_t cnt = v.counts[0];
  GRID_STRIDE(idx, cnt) {
    const uint32_t j = v.vlist[idx];
    if (v.vmis[idx]) {
      const uint64_t r = atomicAdd((unsigned long long*)&v.counts[1], 1ull);
      const uint64_t ts = a.tx.tstart[a.lv.text[j]];
      const uint64_t lb = v.vbest[idx] + 1;
      v.rlist[r] = j;
      v.rlb[r] = lb > ts ? lb : ts;
    } else {
      a.k.lm[j] = v.vbest[idx];
    }
  }
}

hipError_t launch_finish(const PhaseArgs& a, const VerifyBufs& v, hipStream_t s) {
  k_finish<<<grid_for(a.lv.c, 256), 256, 0, s>>>(a, v);
  return hipGetLastError();
}

// Exact fallback after a collision: one wave per key walks positions
// lb, lb+1, ... up to the key's own start, fingerprints each window, and
// verifies hits in increasing order; the first verified hit is the leftmost
// occurrence (no true occurrence lies before lb, see the file header of
// bt_host.cpp).  The key's own start always verifies, so the walk ends.
__global__ __launch_bounds__(256) void k_retry(PhaseArgs a, VerifyBufs v) {
  const uint64_t cnt = v.counts[1];
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const int lane = lane_id();
  for (uint64_t idx = gw; idx < cnt; idx += nw) {
    const uint32_t j = v.rlist[idx];
    const uint64_t lb = v.rlb[idx];
    const uint64_t pos = a.lv.st[j];
    const uint64_t L = a.k.len[j];
    const uint64_t fpk = a.k.fp[j];
    const uint64_t salt = a.tx.tsalt[a.lv.text[j]];
    const uint64_t xp = pow61(a.x, L);
    uint64_t found = pos;
    bool done = false;
    for (uint64_t p0 = lb; p0 <= pos && !done; p0 += 64) {
      const uint64_t p = p0 + lane;
      const bool m = p <= pos && finish_fp(win61_any(a, p, L, xp), salt, a.fpmask) == fpk;
      uint64_t bal = __ballot(m);
      while (bal) {
        const uint64_t q = p0 + (uint64_t)(__ffsll((unsigned long long)bal) - 1);
        bool diff = false;
        for (uint64_t off = 0; off < L && !diff; off += kVChunk) {
          const uint64_t end = L - off < kVChunk ? L : off + kVChunk;
          diff = wave_bytes_differ(a.T, q, pos, off, end);
        }
        if (!diff) {
          found = q;
          done = true;
          break;
        }
        bal &= bal - 1;
      }
    }
    if (lane == 0) a.k.lm[j] = found;
  }
}

hipError_t launch_retry(const PhaseArgs& a, const VerifyBufs& v, hipStream_t s) {
  const unsigned grid = grid_for(a.lv.c * 64, 256, 1024);
  k_retry<<<grid, 256, 0, s>>>(a, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------- marks (a5)

__global__ void k_mark(PhaseArgs a, uint8_t* marked) {
  const LevelDev lv = a.lv;
  GRID_STRIDE(j, lv.c) {
    bool m = a.k.slot[j] != kNoKey && a.k.lm[j] == lv.st[j];
    if (j > 0 && a.k.slot[j - 1] != kNoKey && a.k.lm[j - 1] == lv.st[j - 1]) m = true;
    const uint32_t r = lv.run[j];
    const bool left = j > 0 && lv.run[j - 1] == r;
    const bool right = j + 1 < lv.c && lv.run[j + 1] == r;
    if (!left && !right) m = true;  // a block with no consecutive neighbour
    marked[j] = m ? 1 : 0;
  }
}

hipError_t launch_mark(const PhaseArgs& a, uint8_t* marked, hipStream_t s) {
  k_mark<<<grid_for(a.lv.c, 256), 256, 0, s>>>(a, marked);
  return hipGetLastError();
}

// The mark of block j (as k_mark): its pair or its left neighbour's pair is
// leftmost, or it has no consecutive neighbour.
__device__ __forceinline__ bool mark_of(const PhaseArgs& a, uint64_t j) {
  const LevelDev& lv = a.lv;
  const auto leftmost = [&](uint64_t q) { return a.k.slot[q] != kNoKey && a.k.lm[q] == lv.st[q]; };
  if (leftmost(j) || (j > 0 && leftmost(j - 1))) return true;
  const uint32_t r = lv.run[j];
  const bool left = j > 0 && lv.run[j - 1] == r;
  const bool right = j + 1 < lv.c && lv.run[j + 1] == r;
  return !left && !right;
}

// After phase 1, in one pass: the marks, the pair facts (as k_pair_facts), the
// unmarked indicator that the pointer ranks scan from, and where the next
// level's runs start.  The children of a maximal group of consecutive marked
// blocks of one run are consecutive blocks of one run, so nrun[j] = 1 exactly
// where such a group starts.
__global__ void k_mark_facts(PhaseArgs a, uint8_t* marked, uint8_t* pf, uint64_t* ucnt,
                             uint64_t* nrun) {
  const LevelDev lv = a.lv;
  GRID_STRIDE(j, lv.c) {
    const bool own = a.k.slot[j] != kNoKey;
    const bool m = mark_of(a, j);
    marked[j] = m ? 1 : 0;
    pf[j] = (own && a.k.lm[j] < lv.st[j]) ? 1 : 0;
    ucnt[j] = m ? 0 : 1;
    nrun[j] = (m && (j == 0 || lv.run[j - 1] != lv.run[j] || !mark_of(a, j - 1))) ? 1 : 0;
  }
}

hipError_t launch_mark_facts(const PhaseArgs& a, uint8_t* marked, uint8_t* pf, uint64_t* ucnt,
                             uint64_t* nrun, hipStream_t s) {
  if (!a.lv.c) return hipSuccess;
  k_mark_facts<<<grid_for(a.lv.c, 256), 256, 0, s>>>(a, marked, pf, ucnt, nrun);
  return hipGetLastError();
}

__global__ void k_unmarked_counts(const uint8_t* marked, uint64_t c, uint64_t* cnt) {
  GRID_STRIDE(j, c) cnt[j] = marked[j] ? 0 : 1;
}

hipError_t launch_unmarked_counts(const uint8_t* marked, uint64_t c, uint64_t* cnt,
                                  hipStream_t s) {
  k_unmarked_counts<<<grid_for(c, 256), 256, 0, s>>>(marked, c, cnt);
  return hipGetLastError();
}

// ---------------------------------------------------------------- pointers (a7)

__global__ void k_pointers(PhaseArgs a, const uint8_t* marked, const uint64_t* uoff,
                           const uint64_t* tfirst, uint64_t* pb, uint64_t* po, uint32_t* err) {
  const LevelDev lv = a.lv;
  GRID_STRIDE(j, lv.c) {
    if (marked[j]) continue;
    const uint64_t p = a.k.lm[j];
    const uint32_t tx = lv.text[j];
    // the target block: the last one starting at or before p, searched among
    // the blocks of j's own text before j (an occurrence lies in its text and
    // ends by j's start; the checks below catch anything else)
    uint64_t lo = tfirst[tx], hi = j;
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (lv.st[mid] <= p) lo = mid; else hi = mid;
    }
    const uint64_t t = lo;
    const uint64_t lj = block_len(lv, a.tx, j), lt = block_len(lv, a.tx, t);
    bool ok = lv.st[t] <= p && p < lv.st[t] + lt && marked[t] && lv.text[t] == tx &&
              p + lj <= lv.st[j];
    if (ok && p + lj > lv.st[t] + lt)
      ok = t + 1 < lv.c && lv.run[t + 1] == lv.run[t] && marked[t + 1];
    if (!ok) *err = 1;
    const uint64_t u = uoff[j];
    pb[u] = t - tfirst[tx];
    po[u] = p - lv.st[t];
  }
}

hipError_t launch_pointers(const PhaseArgs& a, const uint8_t* marked, const uint64_t* uoff,
                           const uint64_t* tfirst, uint64_t* ptr_block, uint64_t* ptr_off,
                           uint32_t* err, hipStream_t s) {
  k_pointers<<<grid_for(a.lv.c, 256), 256, 0, s>>>(a, marked, uoff, tfirst, ptr_block, ptr_off,
                                                    err);
  return hipGetLastError();
}

// ---------------------------------------------------------------- split (a8)

__global__ void k_child_counts(LevelDev lv, TextsDev tx, const uint8_t* marked, uint64_t bn,
                               uint64_t* cnt) {
  GRID_STRIDE(j, lv.c) {
    cnt[j] = marked[j] ? (block_len(lv, tx, j) + bn - 1) / bn : 0;
  }
}

hipError_t launch_child_counts(const LevelDev& lv, const TextsDev& tx, const uint8_t* marked,
                               uint64_t bn, uint64_t* cnt, hipStream_t s) {
  k_child_counts<<<grid_for(lv.c, 256), 256, 0, s>>>(lv, tx, marked, bn, cnt);
  return hipGetLastError();
}

__global__ void k_text_counts(uint32_t T, const uint64_t* cs, const uint64_t* tfirst,
                              const uint64_t* tcount, const uint64_t* enter, uint64_t* ncount) {
  GRID_STRIDE(t, T) {
    const uint64_t f = tfirst[t];
    ncount[t] = cs[f + tcount[t]] - cs[f] + (enter ? enter[t] : 0);
  }
}

hipError_t launch_text_counts(uint32_t T, const uint64_t* cs, const uint64_t* tfirst,
                              const uint64_t* tcount, const uint64_t* enter, uint64_t* ncount,
                              hipStream_t s) {
  k_text_counts<<<grid_for(T, 256), 256, 0, s>>>(T, cs, tfirst, tcount, enter, ncount);
  return hipGetLastError();
}

__global__ void k_write_children(LevelDev lv, TextsDev tx, const uint8_t* marked, uint64_t bn,
                                 const uint64_t* cs, const uint64_t* tfirst,
                                 const uint64_t* ntfirst, uint64_t* nst, uint32_t* ntext) {
  GRID_STRIDE(j, lv.c) {
    if (!marked[j]) continue;
    const uint32_t t = lv.text[j];
    const uint64_t base = ntfirst[t] + (cs[j] - cs[tfirst[t]]);
    const uint64_t nk = cs[j + 1] - cs[j];
    const uint64_t st = lv.st[j];
    for (uint64_t k = 0; k < nk; ++k) {
      nst[base + k] = st + k * bn;
      ntext[base + k] = t;
    }
  }
}

hipError_t launch_write_children(const LevelDev& lv, const TextsDev& tx, const uint8_t* marked,
                                 uint64_t bn, uint32_t tau, const uint64_t* cs,
                                 const uint64_t* tfirst, const uint64_t* ntfirst, uint64_t* nst,
                                 uint32_t* ntext, hipStream_t s) {
  (void)tau;
  k_write_children<<<grid_for(lv.c, 256), 256, 0, s>>>(lv, tx, marked, bn, cs, tfirst, ntfirst,
                                                        nst, ntext);
  return hipGetLastError();
}

__global__ void k_write_entering(const uint32_t* ids, TextsDev tx, uint64_t bn,
                                 const uint64_t* ntfirst, uint64_t* nst, uint32_t* ntext) {
  const uint32_t t = ids[blockIdx.x];
  const uint64_t ts = tx.tstart[t], te = tx.tend[t];
  const uint64_t nb = (te - ts + bn - 1) / bn;
  const uint64_t base = ntfirst[t];
  for (uint64_t k = threadIdx.x; k < nb; k += blockDim.x) {
    nst[base + k] = ts + k * bn;
    ntext[base + k] = t;
  }
}

hipError_t launch_write_entering(const uint32_t* ids, uint32_t E, const TextsDev& tx,
                                 uint64_t bn, const uint64_t* ntfirst, uint64_t* nst,
                                 uint32_t* ntext, hipStream_t s) {
  if (!E) return hipSuccess;
  k_write_entering<<<E, 256, 0, s>>>(ids, tx, bn, ntfirst, nst, ntext);
  return hipGetLastError();
}

__global__ void k_run_flags(const uint64_t* st, const uint32_t* text, uint64_t c, uint64_t b,
                            uint64_t* rflag) {
  GRID_STRIDE(j, c) {
    rflag[j] = (j == 0 || text[j] != text[j - 1] || st[j] != st[j - 1] + b) ? 1 : 0;
  }
}

hipError_t launch_run_flags(const uint64_t* st, const uint32_t* text, uint64_t c, uint64_t b,
                            uint64_t* rflag, hipStream_t s) {
  k_run_flags<<<grid_for(c, 256), 256, 0, s>>>(st, text, c, b, rflag);
  return hipGetLastError();
}

__global__ void k_run_table(const uint64_t* st, const uint32_t* text, uint64_t c, uint64_t b,
                            TextsDev tx, const uint64_t* roff, uint32_t* run, uint64_t* rs,
                            uint64_t* re, uint32_t* rtext) {
  GRID_STRIDE(j, c) {
    const uint64_t r = roff[j + 1] - 1;
    run[j] = (uint32_t)r;
    if (roff[j + 1] != roff[j]) {
      rs[r] = st[j];
      rtext[r] = text[j];
    }
    const bool last = (j + 1 == c) || (roff[j + 2] != roff[j + 1]);
    if (last) {
      const uint64_t te = tx.tend[text[j]];
      re[r] = st[j] + (te - st[j] < b ? te - st[j] : b);
    }
  }
}

hipError_t launch_run_table(const uint64_t* st, const uint32_t* text, uint64_t c, uint64_t b,
                            const TextsDev& tx, const uint64_t* roff, uint32_t* run,
                            uint64_t* rs, uint64_t* re, uint32_t* rtext, hipStream_t s) {
  k_run_table<<<grid_for(c, 256), 256, 0, s>>>(st, text, c, b, tx, roff, run, rs, re, rtext);
  return hipGetLastError();
}

// ---------------------------------------------------------------- outputs

__global__ void k_pack_marks(const uint8_t* marked, uint32_t T, const uint64_t* tfirst,
                             const uint64_t* tcount, const uint64_t* woff, uint64_t nwords,
                             uint64_t* words) {
  GRID_STRIDE(wi, nwords) {
    uint64_t lo = 0, hi = T;
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (woff[mid] <= wi) lo = mid; else hi = mid;
    }
    // skip texts with no words (equal offsets): take the last one not past wi
    const uint64_t t = lo;
    const uint64_t lw = wi - woff[t];
    const uint64_t f = tfirst[t], cnt = tcount[t];
    uint64_t word = 0;
    for (uint64_t k = 0; k < 64; ++k) {
      const uint64_t j = lw * 64 + k;
      if (j < cnt && marked[f + j]) word |= 1ull << k;
    }
    words[wi] = word;
  }
}

hipError_t launch_pack_marks(const uint8_t* marked, uint32_t T, const uint64_t* tfirst,
                             const uint64_t* tcount, const uint64_t* woff, uint64_t nwords,
                             uint64_t* words, hipStream_t s) {
  if (!nwords) return hipSuccess;
  k_pack_marks<<<grid_for(nwords, 256), 256, 0, s>>>(marked, T, tfirst, tcount, woff, nwords,
                                                      words);
  return hipGetLastError();
}

// Leaf bytes: block j of the last level lands at j*b (texts' regions are
// contiguous; only a text-final block is short, and it ends its region; the
// bytes after its end are written as zeros).  Thread k writes output bytes
// [16k, 16k + 16) with one 16-byte store (the last, partial chunk byte by
// byte).  A chunk inside one block, with 24 bytes of the buffer after its
// source, is read as three aligned 8-byte words; any other chunk byte by byte.
__global__ void k_leaves(const uint8_t* __restrict__ T, LevelDev lv, TextsDev tx,
                         uint8_t* __restrict__ out) {
  const uint64_t total = lv.c * lv.b;
  const uint64_t end = tx.tend[tx.T - 1];  // the buffer's end (texts are in order)
  GRID_STRIDE(k, (total + 15) / 16) {
    const uint64_t p = 16 * k;
    uint64_t j = p / lv.b, r = p - j * lv.b;
    uint64_t len = block_len(lv, tx, j), src = lv.st[j];
    uint64_t lo = 0, hi = 0;
    if (r + 16 <= len && src + r + 24 <= end) {
      bytes16_at(T, end, src + r, lo, hi);
    } else {
      for (int e = 0; e < 16 && p + e < total; ++e) {
        if (r == lv.b) {
          ++j;
          r = 0;
          len = block_len(lv, tx, j);
          src = lv.st[j];
        }
        const uint64_t v = r < len ? T[src + r] : 0;
        (e < 8 ? lo : hi) |= v << (8 * (e & 7));
        ++r;
      }
    }
    if (p + 16 <= total) {
      uint4 w;
      w.x = (uint32_t)lo;
      w.y = (uint32_t)(lo >> 32);
      w.z = (uint32_t)hi;
      w.w = (uint32_t)(hi >> 32);
      *reinterpret_cast<uint4*>(out + p) = w;
    } else {
      for (uint64_t e = 0; p + e < total; ++e) out[p + e] = (uint8_t)((e < 8 ? lo : hi) >> (8 * (e & 7)));
    }
  }
}

hipError_t launch_leaves(const uint8_t* T, const LevelDev& lv, const TextsDev& tx, uint8_t* out,
                         hipStream_t s) {
  if (!lv.c) return hipSuccess;
  k_leaves<<<grid_for((lv.c * lv.b + 15) / 16, 256), 256, 0, s>>>(T, lv, tx, out);
  return hipGetLastError();
}

}  // namespace bt
