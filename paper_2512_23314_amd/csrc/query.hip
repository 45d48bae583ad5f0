// Queries on a finished tree (Section 1: access, rank, select) and small
// auxiliary kernels of the build.
//
// access(i): start in level-1 block i / b1 at offset i mod b1.  In a marked
// block move to the child that holds the offset (its index is tau times the
// number of marked blocks before it, plus the child number).  In an unmarked
// block follow the pointer (t, off): the content continues at offset off + o
// of block t, or of block t+1 when that passes the end of t; both are marked,
// so the walk then descends from there.  At the last level read the leaf byte.
#include "common.hpp"
#include "internal.hpp"
#include "query.hpp"

namespace bt {

static unsigned grid_for(uint64_t n, unsigned threads, unsigned cap = 8192) {
  uint64_t g = (n + threads - 1) / threads;
  if (g == 0) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

#define GRID_STRIDE(i, n)                                                        \
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
       i += (uint64_t)gridDim.x * blockDim.x)

__device__ __forceinline__ uint64_t marks_before(const QLevel& L, uint64_t j) {
  const uint64_t w = L.words[j >> 6];
  const uint64_t below = (j & 63) ? (w << (64 - (j & 63))) : 0;
  return L.wrank[j >> 6] + __popcll(below);
}
__device__ __forceinline__ bool is_marked(const QLevel& L, uint64_t j) {
  return (L.words[j >> 6] >> (j & 63)) & 1;
}

// Descend from level 0 to the leaf holding text position i.  Returns the leaf
// index and the offset inside it.  Calls on_ptr(level, j, u, t, off, o) at every
// pointer that is followed (for rank's counter adjustments).
template <typename F>
__device__ __forceinline__ void descend(const QTree& q, uint64_t i, uint64_t& leaf, uint64_t& off,
                                        F&& on_ptr) {
  const QLevel* lv = q.lv;
  uint64_t j = i / lv[0].b;
  uint64_t o = i - j * lv[0].b;
  uint32_t l = 0;
  while (l + 1 < q.h) {
    const QLevel L = lv[l];
    const uint64_t r1 = marks_before(L, j);
    if (is_marked(L, j)) {
      const uint64_t bn = lv[l + 1].b;
      const uint64_t k = o / bn;
      j = r1 * q.tau + k;
      o -= k * bn;
      ++l;
    } else {
      const uint64_t u = j - r1;
      uint64_t t = L.pb[u];
      uint64_t o2 = L.po[u] + o;
      on_ptr(l, j, u, t, L.po[u], o);
      if (o2 >= L.b) {
        o2 -= L.b;
        ++t;
      }
      j = t;
      o = o2;
    }
  }
  leaf = j;
  off = o;
}

__global__ void k_access(QTree q, const uint64_t* __restrict__ pos, uint64_t m,
                         uint8_t* __restrict__ out, uint32_t* bad) {
  GRID_STRIDE(k, m) {
    const uint64_t i = pos[k];
    if (i >= q.n) {
      out[k] = 0;
      *bad = 1;
      continue;
    }
    uint64_t leaf, o;
    descend(q, i, leaf, o, [](uint32_t, uint64_t, uint64_t, uint64_t, uint64_t, uint64_t) {});
    out[k] = q.leaves[leaf * q.leaf_len + o];
  }
}

hipError_t launch_access(QTree t, const uint64_t* pos, uint64_t m, uint8_t* out, uint32_t* bad,
                         hipStream_t s) {
  if (!m) return hipSuccess;
  k_access<<<grid_for(m, 256), 256, 0, s>>>(t, pos, m, out, bad);
  return hipGetLastError();
}

// Counter of width w at index idx.
__device__ __forceinline__ uint64_t narrow_at(const uint8_t* p, uint32_t w, uint64_t idx) {
  return w == 1 ? p[idx]
                : w == 2 ? reinterpret_cast<const uint16_t*>(p)[idx]
                         : reinterpret_cast<const uint32_t*>(p)[idx];
}

// R (occurrences of symbol s before block x of level l, from the text's
// start): relative counts up the parents to the nearest absolute level.
__device__ uint64_t block_count(const QTree& q, uint32_t l, uint64_t x, uint32_t s) {
  uint64_t r = 0;
  while (!q.lv[l].acnt) {
    const QLevel& L = q.lv[l];
    r += narrow_at(L.qc, L.qw, x * q.S + s);
    x = q.lv[l - 1].msel[x / q.tau];
    --l;
  }
  return r + q.lv[l].acnt[x * q.S + s];
}

// R of block jc of level l1 whose parent has R = rp.
__device__ __forceinline__ uint64_t child_count(const QTree& q, uint32_t l1, uint64_t jc, uint32_t s,
                                                uint64_t rp) {
  const QLevel& N = q.lv[l1];
  return N.acnt ? N.acnt[jc * q.S + s] : rp + narrow_at(N.qc, N.qw, jc * q.S + s);
}

// rank(c, i): the walk of access, carrying R of the current block.  Every
// pointer followed from block j (unmarked number u, target t) adds
// R[j] - (R[t] + P[u]), the count before block j minus the count before the
// source position; at the leaf, R of the leaf and the bytes before the offset.
__global__ void k_rank(QTree q, const uint8_t* __restrict__ cs, const uint64_t* __restrict__ pos,
                       uint64_t m, uint64_t* __restrict__ out) {
  const uint32_t S = q.S;
  GRID_STRIDE(k, m) {
    const uint64_t i = pos[k];
    const uint8_t ch = cs[k];
    const int s = q.sym[ch];
    if (i > q.n) {
      out[k] = ~0ull;
      continue;
    }
    if (s < 0) {
      out[k] = 0;
      continue;
    }
    if (i == q.n) {
      out[k] = q.total[s];
      continue;
    }
    const QLevel* lv = q.lv;
    uint64_t j = i / lv[0].b;
    uint64_t o = i - j * lv[0].b;
    uint64_t R = lv[0].acnt[j * S + s];
    int64_t acc = 0;
    uint32_t l = 0;
    while (l + 1 < q.h) {
      const QLevel& L = lv[l];
      const uint64_t r1 = marks_before(L, j);
      if (is_marked(L, j)) {
        const uint64_t bn = lv[l + 1].b;
        const uint64_t x = o / bn;
        j = r1 * q.tau + x;
        o -= x * bn;
        ++l;
        R = child_count(q, l, j, s, R);
      } else {
        const uint64_t u = j - r1;
        uint64_t t = L.pb[u];
        uint64_t o2 = L.po[u] + o;
        const uint64_t Rt = block_count(q, l, t, s);
        acc += (int64_t)R - (int64_t)(Rt + narrow_at(L.pc, L.pw, u * S + s));
        if (o2 >= L.b) {
          o2 -= L.b;
          ++t;
          R = block_count(q, l, t, s);
        } else {
          R = Rt;
        }
        j = t;
        o = o2;
      }
    }
    acc += (int64_t)R;
    const uint8_t* lb = q.leaves + j * q.leaf_len;
    for (uint64_t r = 0; r < o; ++r) acc += lb[r] == ch;
    out[k] = (uint64_t)acc;
  }
}

hipError_t launch_rank(QTree t, const uint8_t* cs, const uint64_t* pos, uint64_t m, uint64_t* out,
                       hipStream_t s) {
  if (!m) return hipSuccess;
  k_rank<<<grid_for(m, 256), 256, 0, s>>>(t, cs, pos, m, out);
  return hipGetLastError();
}

// select(c, k): keep the invariant R[j] < k <= R[j] + (occurrences in block
// j), carrying R of the current block.  Level 1: binary search over the blocks.
// Marked block: the last child whose count is below k.  Unmarked block j with
// pointer (t, off): the wanted occurrence is the (k - R[j])-th inside the block,
// i.e. occurrence k' = R[t] + P[u] + (k - R[j]) of the source, which lies in
// block t or t+1; the answer moves by (start of j) - (source position).  At the
// leaf, scan its bytes.
__global__ void k_select(QTree q, const uint8_t* __restrict__ cs, const uint64_t* __restrict__ ks,
                         uint64_t m, uint64_t* __restrict__ out) {
  const uint32_t S = q.S;
  GRID_STRIDE(qi, m) {
    const uint8_t ch = cs[qi];
    uint64_t k = ks[qi];
    const int s = q.sym[ch];
    if (s < 0 || k == 0 || k > q.total[s]) {
      out[qi] = ~0ull;
      continue;
    }
    const QLevel* lv = q.lv;
    uint64_t lo = 0, hi = lv[0].c;
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (lv[0].acnt[mid * S + s] < k) lo = mid; else hi = mid;
    }
    uint64_t j = lo;
    uint64_t R = lv[0].acnt[j * S + s];
    uint32_t l = 0;
    uint64_t shift = 0;
    while (l + 1 < q.h) {
      const QLevel& L = lv[l];
      const uint64_t r1 = marks_before(L, j);
      if (is_marked(L, j)) {
        const QLevel& N = lv[l + 1];
        const uint64_t j0 = r1 * q.tau;
        uint64_t nch = N.c - j0;
        if (nch > q.tau) nch = q.tau;
        // the first child starts where its parent does: its R is the parent's
        uint64_t x = 1, Rx = R;
        while (x < nch) {
          const uint64_t Rn = child_count(q, l + 1, j0 + x, s, R);
          if (Rn >= k) break;
          Rx = Rn;
          ++x;
        }
        j = j0 + x - 1;
        R = Rx;
        ++l;
      } else {
        const uint64_t u = j - r1;
        const uint64_t t = L.pb[u];
        const uint64_t src = L.st[t] + L.po[u];
        const uint64_t Rt = block_count(q, l, t, s);
        const uint64_t k2 = Rt + narrow_at(L.pc, L.pw, u * S + s) + (k - R);
        shift += L.st[j] - src;
        uint64_t nt = t, Rn = Rt;
        if (t + 1 < L.c && L.st[t + 1] == L.st[t] + L.b) {
          const uint64_t R1 = block_count(q, l, t + 1, s);
          if (R1 < k2) {
            nt = t + 1;
            Rn = R1;
          }
        }
        j = nt;
        k = k2;
        R = Rn;
      }
    }
    const QLevel& LH = lv[q.h - 1];
    uint64_t need = k - R;
    const uint8_t* lb = q.leaves + j * q.leaf_len;
    uint64_t res = ~0ull;
    const uint64_t rest = q.tstart + q.n - LH.st[j];
    const uint64_t llen = rest < q.leaf_len ? rest : q.leaf_len;
    for (uint64_t o = 0; o < llen; ++o) {
      if (lb[o] == ch && --need == 0) {
        res = LH.st[j] + o + shift - q.tstart;
        break;
      }
    }
    out[qi] = res;
  }
}

hipError_t launch_select(QTree t, const uint8_t* cs, const uint64_t* ks, uint64_t m, uint64_t* out,
                         hipStream_t s) {
  if (!m) return hipSuccess;
  k_select<<<grid_for(m, 256), 256, 0, s>>>(t, cs, ks, m, out);
  return hipGetLastError();
}

__global__ void k_rank_empty(const uint64_t* pos, uint64_t m, uint64_t* out) {
  GRID_STRIDE(k, m) out[k] = pos[k] == 0 ? 0 : ~0ull;
}

hipError_t launch_rank_empty(const uint64_t* pos, uint64_t m, uint64_t* out, hipStream_t s) {
  if (!m) return hipSuccess;
  k_rank_empty<<<grid_for(m, 256), 256, 0, s>>>(pos, m, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- auxiliary

// Each thread keeps its own 256-bit set in LDS column t (word k of thread t at
// s[k][t]: a wave's lanes touch 64 different banks); 16 bytes per load.  The
// columns are then ORed and merged into the global set, which is read first so
// that most workgroups skip the atomic.
__global__ __launch_bounds__(256) void k_byte_presence(const uint8_t* __restrict__ T, uint64_t n,
                                                       uint32_t* __restrict__ seen) {
  __shared__ uint32_t s[8][256];
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 8; ++k) s[k][t] = 0;
  const auto add = [&](uint32_t c) { atomicOr(&s[c >> 5][t], 1u << (c & 31)); };
  const uint64_t mis = reinterpret_cast<uintptr_t>(T) & 15;
  const uint64_t head = mis ? (16 - mis < n ? 16 - mis : n) : 0;
  const uint64_t body = (n - head) / 16;
  const uint4* __restrict__ B = reinterpret_cast<const uint4*>(T + head);
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + t; i < body; i += (uint64_t)gridDim.x * 256) {
    const uint4 v = B[i];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int k = 0; k < 4; ++k) add((w[q] >> (8 * k)) & 0xFFu);
  }
  if (blockIdx.x == 0) {
    for (uint64_t i = t; i < head; i += 256) add(T[i]);
    for (uint64_t i = head + body * 16 + t; i < n; i += 256) add(T[i]);
  }
  __syncthreads();
  // word k = t / 32 over the 256 columns: eight per lane, then 32 lanes
  const int k = t >> 5, part = t & 31;
  uint32_t m = 0;
#pragma unroll
  for (int e = 0; e < 8; ++e) m |= s[k][part * 8 + e];
#pragma unroll
  for (int d = 16; d >= 1; d >>= 1) m |= __shfl_xor(m, d);
  if (part == 0 && m && (seen[k] | m) != seen[k]) atomicOr(&seen[k], m);
}

hipError_t launch_byte_presence(const uint8_t* T, uint64_t n, uint32_t* seen, hipStream_t s) {
  if (!n) return hipSuccess;
  k_byte_presence<<<grid_for((n + 15) / 16, 256, 1024), 256, 0, s>>>(T, n, seen);
  return hipGetLastError();
}

__global__ void k_last_block_len(LevelDev lv, TextsDev tx, const uint64_t* tfirst,
                                 const uint64_t* tcount, uint64_t* out) {
  GRID_STRIDE(t, tx.T) {
    if (!tcount[t]) {
      out[t] = 0;
      continue;
    }
    const uint64_t j = tfirst[t] + tcount[t] - 1;
    const uint64_t st = lv.st[j], te = tx.tend[t];
    out[t] = te - st < lv.b ? te - st : lv.b;
  }
}

hipError_t launch_last_block_len(const LevelDev& lv, const TextsDev& tx, const uint64_t* tfirst,
                                 const uint64_t* tcount, uint64_t* out, hipStream_t s) {
  k_last_block_len<<<grid_for(tx.T, 256), 256, 0, s>>>(lv, tx, tfirst, tcount, out);
  return hipGetLastError();
}

__global__ void k_text_deltas(const uint64_t* scanned, const uint64_t* tfirst,
                              const uint64_t* tcount, uint32_t T, uint64_t* out) {
  GRID_STRIDE(t, T) out[t] = scanned[tfirst[t] + tcount[t]] - scanned[tfirst[t]];
}

hipError_t launch_text_deltas(const uint64_t* scanned, const uint64_t* tfirst,
                              const uint64_t* tcount, uint32_t T, uint64_t* out, hipStream_t s) {
  k_text_deltas<<<grid_for(T, 256), 256, 0, s>>>(scanned, tfirst, tcount, T, out);
  return hipGetLastError();
}

__global__ void k_word_pop(const uint64_t* words, uint64_t nwords, uint64_t* out) {
  GRID_STRIDE(w, nwords) out[w] = __popcll(words[w]);
}

hipError_t launch_word_pop(const uint64_t* words, uint64_t nwords, uint64_t* out, hipStream_t s) {
  if (!nwords) return hipSuccess;
  k_word_pop<<<grid_for(nwords, 256), 256, 0, s>>>(words, nwords, out);
  return hipGetLastError();
}

// wrank[w] = marks in words [first word of w's text, w)
__global__ void k_word_rank(const uint64_t* scanned, uint32_t T, const uint64_t* woff,
                            uint64_t nwords, uint64_t* wrank) {
  GRID_STRIDE(w, nwords) {
    uint64_t lo = 0, hi = T;
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (woff[mid] <= w) lo = mid; else hi = mid;
    }
    wrank[w] = scanned[w] - scanned[woff[lo]];
  }
}

hipError_t launch_word_rank(const uint64_t* scanned, uint32_t T, const uint64_t* woff,
                            uint64_t nwords, uint64_t* wrank, hipStream_t s) {
  if (!nwords) return hipSuccess;
  k_word_rank<<<grid_for(nwords, 256), 256, 0, s>>>(scanned, T, woff, nwords, wrank);
  return hipGetLastError();
}

}  // namespace bt
