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

// ---------------------------------------------------------------- auxiliary

__global__ void k_histogram(const uint8_t* __restrict__ T, uint64_t n, uint64_t* hist) {
  __shared__ uint32_t h[256];
  for (int k = threadIdx.x; k < 256; k += blockDim.x) h[k] = 0;
  __syncthreads();
  GRID_STRIDE(i, n) atomicAdd(&h[T[i]], 1u);
  __syncthreads();
  for (int k = threadIdx.x; k < 256; k += blockDim.x)
    if (h[k]) atomicAdd((unsigned long long*)&hist[k], (unsigned long long)h[k]);
}

hipError_t launch_histogram(const uint8_t* T, uint64_t n, uint64_t* hist, hipStream_t s) {
  if (!n) return hipSuccess;
  k_histogram<<<grid_for(n, 256, 2048), 256, 0, s>>>(T, n, hist);
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
