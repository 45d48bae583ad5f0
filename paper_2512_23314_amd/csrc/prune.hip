// Optional pruning (Section 4.1, the phase after marking and pointers).
//
// Runs after every level is built, from the deepest internal level up.  The
// paper states the rule in one paragraph: marked blocks that no pointer
// targets are removed.  The reading implemented here: a marked block j becomes
// a pointer to its leftmost occurrence p on the level when
//   (i)   no pointer of the level targets it, counting those pruning makes,
//   (ii)  none of its children is marked (children that are leaves count as
//         unmarked),
//   (iii) p + |B_j| <= st_j (an occurrence reaching into B_j would need B_j to
//         stay marked), and
//   (iv)  the occurrence lies in one block or in two consecutive blocks;
// its children then leave the level below.  Within a level blocks are judged
// from right to left; a pointer only targets blocks to its left, so a block is
// judged after everything that can target it.
//
// In parallel.  Every block's leftmost occurrence on the level comes from the
// build (phase 2 over all blocks).  Candidates are the marked blocks that pass
// every test except the one against pointers made by pruning.  A candidate's
// own pointer can hit another candidate only through an occurrence that spans
// two blocks (an occurrence inside one block that has an earlier copy has an
// earlier copy itself), so the decision graph is sparse: candidate j -> the
// candidates among its one or two targets, all to its left.  j is pruned iff
// no pruned candidate targets it.  Rounds settle that from the right: a
// candidate whose sources have all been kept is pruned, its targets are kept,
// and a kept candidate releases its own targets.  The rightmost open candidate
// has only settled sources, so every round settles at least one.
#include "common.hpp"
#include "internal.hpp"

namespace bt {

static unsigned grid_of(uint64_t n, unsigned threads = 256, unsigned cap = 8192) {
  uint64_t g = (n + threads - 1) / threads;
  if (g == 0) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

#define PRUNE_STRIDE(i, n)                                                        \
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
       i += (uint64_t)gridDim.x * blockDim.x)

constexpr uint64_t kSpill = 1ull << 63;

__device__ __forceinline__ uint64_t blen(const LevelDev& lv, const TextsDev& tx, uint64_t j) {
  const uint64_t st = lv.st[j];
  const uint64_t te = tx.tend[lv.text[j]];
  return te - st < lv.b ? te - st : lv.b;
}

// The block holding position p (block starts increase across the level).
__device__ __forceinline__ uint64_t block_at(const LevelDev& lv, uint64_t p) {
  uint64_t lo = 0, hi = lv.c;
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) >> 1;
    if (lv.st[mid] <= p) lo = mid; else hi = mid;
  }
  return lo;
}

// Targets of the level's pointers (every unmarked block points at its leftmost
// occurrence).
__global__ void k_prune_targets(PruneDev d) {
  const LevelDev& lv = d.lv;
  PRUNE_STRIDE(j, lv.c) {
    if (d.marked[j]) continue;
    const uint64_t p = d.lm[j];
    const uint64_t t = block_at(lv, p);
    d.tgt[t] = 1;
    if (p + blen(lv, d.tx, j) > lv.st[t] + blen(lv, d.tx, t) && t + 1 < lv.c) d.tgt[t + 1] = 1;
  }
}

__global__ void k_prune_candidates(PruneDev d) {
  const LevelDev& lv = d.lv;
  PRUNE_STRIDE(j, lv.c) {
    uint8_t s = kPruneNot;
    d.pending[j] = 0;
    if (d.marked[j] && !d.tgt[j]) {
      const uint64_t p = d.lm[j], len = blen(lv, d.tx, j), st = lv.st[j];
      if (p + len <= st) {
        const uint64_t t = block_at(lv, p);
        const bool spill = p + len > lv.st[t] + blen(lv, d.tx, t);
        const bool fits = !spill || (t + 1 < lv.c && lv.run[t + 1] == lv.run[t] &&
                                     p + len <= lv.st[t + 1] + blen(lv, d.tx, t + 1));
        if (fits) {
          if (!d.marked[t] || (spill && !d.marked[t + 1]) || lv.text[t] != lv.text[j]) {
            *d.err = 1;  // the level's leftmost occurrences break the lemma
          } else {
            bool inner = false;
            if (d.cmarked) {
              const uint32_t x = lv.text[j];
              const uint64_t base = d.ctfirst[x] + (d.cs[j] - d.cs[d.tfirst[x]]);
              const uint64_t n = d.cs[j + 1] - d.cs[j];
              for (uint64_t k = 0; k < n && !inner; ++k) inner = d.cmarked[base + k] != 0;
            }
            if (!inner) {
              s = kPruneOpen;
              d.tinfo[j] = t | (spill ? kSpill : 0);
            }
          }
        }
      }
    }
    d.state[j] = s;
  }
}

// pending[x] = open candidates that target x
__global__ void k_prune_edges(PruneDev d) {
  PRUNE_STRIDE(j, d.lv.c) {
    if (d.state[j] != kPruneOpen) continue;
    const uint64_t t = d.tinfo[j] & ~kSpill;
    if (d.state[t] == kPruneOpen) atomicAdd(&d.pending[t], 1u);
    if ((d.tinfo[j] & kSpill) && d.state[t + 1] == kPruneOpen) atomicAdd(&d.pending[t + 1], 1u);
  }
}

// Round, first half: open candidates with no unsettled source are pruned and
// keep their open targets.  A target of an open candidate has pending >= 1
// here, so no thread prunes a block that another thread marks kept.
__global__ void k_prune_round_a(PruneDev d) {
  if (blockIdx.x == 0 && threadIdx.x == 0) d.counters[0] = 0;
  PRUNE_STRIDE(j, d.lv.c) {
    if (d.state[j] != kPruneOpen || d.pending[j] != 0) continue;
    d.state[j] = kPrunePruned;
    const uint64_t t = d.tinfo[j] & ~kSpill;
    if (d.state[t] == kPruneOpen) d.state[t] = kPruneKept;
    if ((d.tinfo[j] & kSpill) && d.state[t + 1] == kPruneOpen) d.state[t + 1] = kPruneKept;
  }
}

// Second half: newly kept candidates release their targets; count the
// candidates still open.
__global__ void k_prune_round_b(PruneDev d) {
  PRUNE_STRIDE(j, d.lv.c) {
    const uint8_t s = d.state[j];
    const bool open = s == kPruneOpen;
    const uint64_t bal = __ballot(open);
    if (open && __ffsll((unsigned long long)bal) - 1 == (int)(threadIdx.x & 63))
      atomicAdd((unsigned long long*)&d.counters[0], (unsigned long long)__popcll(bal));
    if (s != kPruneKept) continue;
    const uint64_t t = d.tinfo[j] & ~kSpill;
    if (d.state[t] == kPruneOpen) atomicSub(&d.pending[t], 1u);
    if ((d.tinfo[j] & kSpill) && d.state[t + 1] == kPruneOpen) atomicSub(&d.pending[t + 1], 1u);
    d.state[j] = kPruneKeptDone;
  }
}

// Pruned blocks lose their mark; their children leave the level below.
__global__ void k_prune_apply(PruneDev d) {
  const LevelDev& lv = d.lv;
  PRUNE_STRIDE(j, lv.c) {
    if (d.state[j] != kPrunePruned) continue;
    d.marked[j] = 0;
    const uint32_t x = lv.text[j];
    const uint64_t base = d.ctfirst[x] + (d.cs[j] - d.cs[d.tfirst[x]]);
    const uint64_t n = d.cs[j + 1] - d.cs[j];
    for (uint64_t k = 0; k < n; ++k) d.cgone[base + k] = 1;
  }
}

hipError_t launch_prune_decide_begin(const PruneDev& d, hipStream_t s) {
  if (!d.lv.c) return hipSuccess;
  const unsigned g = grid_of(d.lv.c);
  k_prune_targets<<<g, 256, 0, s>>>(d);
  k_prune_candidates<<<g, 256, 0, s>>>(d);
  k_prune_edges<<<g, 256, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_prune_round(const PruneDev& d, hipStream_t s) {
  const unsigned g = grid_of(d.lv.c);
  k_prune_round_a<<<g, 256, 0, s>>>(d);
  if (d.lv.c) k_prune_round_b<<<g, 256, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_prune_apply(const PruneDev& d, hipStream_t s) {
  if (!d.lv.c) return hipSuccess;
  k_prune_apply<<<grid_of(d.lv.c), 256, 0, s>>>(d);
  return hipGetLastError();
}

// ---- compaction of the level below

// keep[i] = 1 for blocks that stay; unmk[i] = 1 for blocks that stay unmarked
__global__ void k_keep_flags(const uint8_t* gone, const uint8_t* marked, uint64_t c, uint64_t* keep,
                             uint64_t* unmk) {
  PRUNE_STRIDE(i, c) {
    const bool k = !gone[i];
    keep[i] = k ? 1 : 0;
    unmk[i] = (k && marked && !marked[i]) ? 1 : 0;
  }
}

hipError_t launch_keep_flags(const uint8_t* gone, const uint8_t* marked, uint64_t c, uint64_t* keep,
                             uint64_t* unmk, hipStream_t s) {
  if (!c) return hipSuccess;
  k_keep_flags<<<grid_of(c), 256, 0, s>>>(gone, marked, c, keep, unmk);
  return hipGetLastError();
}

// Kept blocks move to their kept rank (kidx, exclusive scan of keep); the
// unmarked ranks (uold, exclusive scan of unmk) move with them, so that the
// compacted level's unmarked ranks need no second scan.
__global__ void k_compact(const CompactDev d) {
  PRUNE_STRIDE(i, d.c + 1) {
    if (i == d.c) {
      d.nuoff[d.kidx[i]] = d.uold[i];
      continue;
    }
    if (d.kidx[i + 1] == d.kidx[i]) continue;
    const uint64_t k = d.kidx[i];
    d.nst[k] = d.st[i];
    d.ntext[k] = d.text[i];
    if (d.marked) d.nmarked[k] = d.marked[i];
    if (d.lm) d.nlm[k] = d.lm[i];
    d.nuoff[k] = d.uold[i];
  }
}

hipError_t launch_compact(const CompactDev& d, hipStream_t s) {
  k_compact<<<grid_of(d.c + 1), 256, 0, s>>>(d);
  return hipGetLastError();
}

// First block of each text after compaction.
__global__ void k_gather_firsts(const uint64_t* kidx, const uint64_t* tfirst, uint32_t T,
                                uint64_t* out) {
  PRUNE_STRIDE(t, T) out[t] = kidx[tfirst[t]];
}

hipError_t launch_gather_firsts(const uint64_t* kidx, const uint64_t* tfirst, uint32_t T,
                                uint64_t* out, hipStream_t s) {
  if (!T) return hipSuccess;
  k_gather_firsts<<<grid_of(T), 256, 0, s>>>(kidx, tfirst, T, out);
  return hipGetLastError();
}

}  // namespace bt
