// Sort-based phases (Section 5.1): the paper's first parallel construction,
// which sorts fingerprints instead of hashing them, as an alternative to the
// probe scan of one phase.
//
// Every scanned window contributes (its fingerprint, its position); then every
// key contributes (its fingerprint, its block marked as a key).  A stable radix
// sort by fingerprint makes equal fingerprints consecutive, with the windows of
// a group first, in position order (they are emitted in position order), and
// the keys last.  The first position of each group is broadcast to the group's
// members through a scan: the scan of the group-head flags numbers the groups,
// each head stores its position under its group number, and every key reads
// the entry of its group (Section 5.1 uses a prefix sum over an occurrence
// array for the same broadcast).  A key then lowers its slot's smallest
// position to that first window.  Resolve, byte verification and retry follow
// as after the probe scan, and every slot ends with the same smallest position
// as there, so the tree is bit-identical.  Windows whose main-length window
// does not fit the run, and blocks without a key, carry a fingerprint above
// every real one, which no key matches.
#include <hipcub/hipcub.hpp>

#include "common.hpp"
#include "internal.hpp"
#include "window.hpp"

namespace bt {

static unsigned sgrid(uint64_t n, unsigned threads = 256, unsigned cap = 8192) {
  uint64_t g = (n + threads - 1) / threads;
  if (g == 0) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

#define SORT_STRIDE(i, n)                                                         \
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
       i += (uint64_t)gridDim.x * blockDim.x)

constexpr uint64_t kKeyBit = 1ull << 63;  // a key's entry: its block, not a position
constexpr uint64_t kSortChunk = 64 * 16;  // windows per wave and chunk

// Windows, numbered segment after segment: in a chunk of 1024 window numbers
// lane l takes chunk + 64k + l, finding its segment once and then walking.
// The text's short final key, if any, is compared directly, as in the scan.
__global__ void k_sort_emit(PhaseArgs a, const uint64_t* __restrict__ woff, uint64_t none,
                            uint64_t* __restrict__ fpv, uint64_t* __restrict__ posv) {
  const uint64_t R = a.lv.R, W = woff[R];
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t lane = threadIdx.x & 63;
  for (uint64_t ch = gw; ch * kSortChunk < W; ch += nw) {
    const uint64_t w0 = ch * kSortChunk + lane;
    if (w0 >= W) continue;
    uint64_t lo = 0, hi = R;
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (woff[mid] <= w0) lo = mid; else hi = mid;
    }
    uint64_t r = lo, wo = woff[r], wn = woff[r + 1];
    for (uint64_t w = w0; w < W && w < (ch + 1) * kSortChunk; w += 64) {
      while (w >= wn) {
        ++r;
        wo = wn;
        wn = woff[r + 1];
      }
      const uint64_t i = a.lv.rs[r] + (w - wo), re = a.lv.re[r];
      const uint32_t t = a.lv.rtext[r];
      const uint64_t salt = a.tx.tsalt[t];
      uint64_t f = none;
      if (i + a.Lmain <= re) f = finish_fp(win61_any(a, i, a.Lmain, a.xLmain), salt, a.fpmask);
      fpv[w] = f;
      posv[w] = i;
      const uint64_t oL = a.odd.L[t];
      if (oL && i + oL <= re && i < a.odd.pos[t]) {
        const uint64_t g = finish_fp(win61_any(a, i, oL, a.odd.xp[t]), salt, a.fpmask);
        if (g == a.odd.fp[t] && i < a.odd.best[t])
          atomicMin((unsigned long long*)&a.odd.best[t], (unsigned long long)i);
      }
    }
  }
}

// Keys after the windows: entry W + j for block j.
__global__ void k_sort_keys(PhaseArgs a, uint64_t W, uint64_t none, uint64_t* __restrict__ fpv,
                            uint64_t* __restrict__ posv) {
  SORT_STRIDE(j, a.lv.c) {
    const uint32_t s = a.k.slot[j];
    const bool key = s != kNoKey && s != kOddKey && s != kCopyKey;
    fpv[W + j] = key ? a.k.fp[j] : none;
    posv[W + j] = kKeyBit | j;
  }
}

__device__ __forceinline__ bool head_at(const uint64_t* fp, uint64_t i) {
  return i == 0 || fp[i] != fp[i - 1];
}

__global__ void k_sort_heads(const uint64_t* __restrict__ fp, uint64_t n, uint64_t* __restrict__ h) {
  SORT_STRIDE(i, n) h[i] = head_at(fp, i) ? 1 : 0;
}

// After the exclusive scan of the head flags (gx): a head's group is gx[i], any
// other element's gx[i] - 1.  gfirst[group] = first window position + 1, or 0
// when the group starts with a key (it then holds no window).
__global__ void k_sort_first(const uint64_t* __restrict__ fp, const uint64_t* __restrict__ pos,
                             const uint64_t* __restrict__ gx, uint64_t n,
                             uint64_t* __restrict__ gfirst) {
  SORT_STRIDE(i, n) {
    if (head_at(fp, i)) gfirst[gx[i]] = (pos[i] & kKeyBit) ? 0 : pos[i] + 1;
  }
}

__global__ void k_sort_keys_best(PhaseArgs a, const uint64_t* __restrict__ fp,
                                 const uint64_t* __restrict__ pos, const uint64_t* __restrict__ gx,
                                 uint64_t n, const uint64_t* __restrict__ gfirst) {
  SORT_STRIDE(i, n) {
    const uint64_t p = pos[i];
    if (!(p & kKeyBit)) continue;
    const uint64_t g = head_at(fp, i) ? gx[i] : gx[i] - 1;
    const uint64_t first = gfirst[g];
    if (!first) continue;
    const uint32_t s = a.k.slot[p & ~kKeyBit];
    if (s == kNoKey || s == kOddKey || s == kCopyKey) continue;
    atomicMin((unsigned long long*)&a.tab.slots[s].best, (unsigned long long)(first - 1));
  }
}

hipError_t launch_sort_emit(const PhaseArgs& a, const uint64_t* woff, uint64_t W, uint64_t none,
                            uint64_t* fpv, uint64_t* posv, hipStream_t s) {
  const uint64_t waves = (W + kSortChunk - 1) / kSortChunk;
  if (W) k_sort_emit<<<sgrid(waves * 64, 256, 4096), 256, 0, s>>>(a, woff, none, fpv, posv);
  if (a.lv.c) k_sort_keys<<<sgrid(a.lv.c), 256, 0, s>>>(a, W, none, fpv, posv);
  return hipGetLastError();
}

hipError_t sort_pairs_u64(void* tmp, size_t& tmp_bytes, const uint64_t* kin, uint64_t* kout,
                          const uint64_t* vin, uint64_t* vout, uint64_t n, int end_bit,
                          hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, kin, kout, vin, vout, (int)n, 0, end_bit,
                                            s);
}

hipError_t launch_sort_heads(const uint64_t* fp, uint64_t n, uint64_t* h, hipStream_t s) {
  if (n) k_sort_heads<<<sgrid(n), 256, 0, s>>>(fp, n, h);
  return hipGetLastError();
}

hipError_t launch_sort_groups(const PhaseArgs& a, const uint64_t* fp, const uint64_t* pos,
                              const uint64_t* gx, uint64_t n, uint64_t* gfirst, hipStream_t s) {
  if (!n) return hipSuccess;
  k_sort_first<<<sgrid(n), 256, 0, s>>>(fp, pos, gx, n, gfirst);
  k_sort_keys_best<<<sgrid(n), 256, 0, s>>>(a, fp, pos, gx, n, gfirst);
  return hipGetLastError();
}

}  // namespace bt
