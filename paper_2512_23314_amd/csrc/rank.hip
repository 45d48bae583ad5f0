// Rank/select support of a block tree (Section 1 defines the queries; the
// counters follow the usual block-tree scheme of storing, per block, how often
// each symbol occurs before it, made compact).  Built from the text during
// construction, only when requested.  Per level l with block length b:
//   R[l][j][s]  occurrences of symbol s in T[text start, start of block j),
//               for every block j (leaves included), stored in one of two forms:
//     absolute  (u32) on a tree's first level, and on levels whose relative
//               counts would need 32 bits anyway;
//     relative  Q[l][j][s] = R[l][j][s] - R[l-1][parent][s], the occurrences
//               inside the parent before the block: at most (tau - 1) b, so 8
//               or 16 bits.  A query recovers R by walking up the parents
//               (msel: the index of each marked block of a level) to the
//               nearest absolute level.
//   P[l][u][s]  occurrences of s in T[start of target block t, source
//               position) for the u-th unmarked block: below b, so 8, 16 or
//               32 bits.
// Symbols are the text's distinct byte values, densely renumbered.
//
// All come from a sampled count table G: G[k][s] = occurrences of s in the
// first k*Q bytes of the concatenation (Q = 1024), so that the count before any
// position p is G[p / Q] plus a histogram of at most Q bytes.  A level's
// absolute counts are formed first (a temporary of 4 B per block and symbol),
// then narrowed.
#include "common.hpp"
#include "internal.hpp"
#include "query.hpp"

namespace bt {

#define GRID_STRIDE(i, n)                                                        \
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
       i += (uint64_t)gridDim.x * blockDim.x)

static unsigned grid_for(uint64_t n, unsigned threads, unsigned cap = 8192) {
  uint64_t g = (n + threads - 1) / threads;
  if (g == 0) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

// ---- the sampled count table

// H[k][s]: occurrences of symbol s in chunk k (bytes [kQ, (k+1)Q) of the range).
__global__ void k_chunk_hist(const uint8_t* __restrict__ T, uint64_t N, const int16_t* sym,
                             uint32_t S, uint64_t K, uint32_t* H) {
  __shared__ uint32_t h[256];
  for (uint64_t k = blockIdx.x; k < K; k += gridDim.x) {
    for (int b = threadIdx.x; b < 256; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const uint64_t base = k * kRankQ;
    for (uint64_t i = threadIdx.x; i < kRankQ && base + i < N; i += blockDim.x)
      atomicAdd(&h[T[base + i]], 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < 256; b += blockDim.x)
      if (sym[b] >= 0) H[k * S + sym[b]] = h[b];
    __syncthreads();
  }
}

constexpr uint64_t kColRows = 1024;  // rows per block of the column scan

// Column sums of H over blocks of kColRows rows: B[blk][s].
__global__ void k_col_block_sums(const uint32_t* H, uint64_t K, uint32_t S, uint64_t* B) {
  const uint64_t blk = blockIdx.x;
  for (uint32_t s = threadIdx.x; s < S; s += blockDim.x) {
    uint64_t sum = 0;
    const uint64_t k0 = blk * kColRows;
    for (uint64_t k = k0; k < k0 + kColRows && k < K; ++k) sum += H[k * S + s];
    B[blk * S + s] = sum;
  }
}

// Exclusive scan of B along blocks (one thread per column).
__global__ void k_col_block_scan(uint64_t* B, uint64_t nblk, uint32_t S) {
  for (uint32_t s = threadIdx.x; s < S; s += blockDim.x) {
    uint64_t run = 0;
    for (uint64_t b = 0; b < nblk; ++b) {
      const uint64_t v = B[b * S + s];
      B[b * S + s] = run;
      run += v;
    }
  }
}

// G[k][s] = exclusive prefix along k; G[K][s] = column total.
__global__ void k_col_scan(const uint32_t* H, uint64_t K, uint32_t S, const uint64_t* B,
                           uint64_t* G) {
  const uint64_t blk = blockIdx.x;
  for (uint32_t s = threadIdx.x; s < S; s += blockDim.x) {
    uint64_t run = B[blk * S + s];
    const uint64_t k0 = blk * kColRows;
    uint64_t k = k0;
    for (; k < k0 + kColRows && k < K; ++k) {
      G[k * S + s] = run;
      run += H[k * S + s];
    }
    if (k == K) G[K * S + s] = run;
  }
}

// ---- counts before a position, one wave per query

// Per-wave LDS: 256 u32 partial counts.
__device__ void wave_counts_before(const RankCtx& rc, uint64_t p, uint32_t* part) {
  const int lane = lane_id();
  const uint64_t row = (p - rc.o0) / kRankQ;
  const uint64_t base = rc.o0 + row * kRankQ;
  for (int b = lane; b < 256; b += 64) part[b] = 0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (uint64_t o = (uint64_t)lane * 16; base + o < p; o += 64 * 16) {
    const uint64_t e = p - (base + o) < 16 ? p - (base + o) : 16;
    for (uint64_t q = 0; q < e; ++q) atomicAdd(&part[rc.T[base + o + q]], 1u);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// value of symbol s before p (after wave_counts_before filled part)
__device__ __forceinline__ uint64_t count_of(const RankCtx& rc, uint64_t p, const uint32_t* part,
                                             uint32_t s) {
  const uint64_t row = (p - rc.o0) / kRankQ;
  return rc.G[row * rc.S + s] + part[rc.byte_of[s]];
}

// Per text: Rt[t][s] = count before the text's start, Rtot[t][s] = in the text.
__global__ __launch_bounds__(256) void k_text_counts(RankCtx rc, TextsDev tx, uint64_t* Rt,
                                                     uint64_t* Rtot) {
  __shared__ uint32_t s_part[4][256];
  uint32_t* part = s_part[threadIdx.x >> 6];
  const int lane = lane_id();
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t t = gw; t < tx.T; t += nw) {
    wave_counts_before(rc, tx.tstart[t], part);
    for (uint32_t s = lane; s < rc.S; s += 64) Rt[t * rc.S + s] = count_of(rc, tx.tstart[t], part, s);
    wave_counts_before(rc, tx.tend[t], part);
    for (uint32_t s = lane; s < rc.S; s += 64)
      Rtot[t * rc.S + s] = count_of(rc, tx.tend[t], part, s) - Rt[t * rc.S + s];
  }
}

// cnt[j][s] for every block of a level.
__global__ __launch_bounds__(256) void k_block_counts(RankCtx rc, const uint64_t* st,
                                                      const uint32_t* text, uint64_t c,
                                                      const uint64_t* Rt, uint32_t* cnt) {
  __shared__ uint32_t s_part[4][256];
  uint32_t* part = s_part[threadIdx.x >> 6];
  const int lane = lane_id();
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t j = gw; j < c; j += nw) {
    const uint64_t p = st[j];
    wave_counts_before(rc, p, part);
    const uint64_t t = text[j];
    for (uint32_t s = lane; s < rc.S; s += 64)
      cnt[j * rc.S + s] = (uint32_t)(count_of(rc, p, part, s) - Rt[t * rc.S + s]);
  }
}

__device__ __forceinline__ void put_narrow(uint8_t* p, uint32_t w, uint64_t idx, uint32_t v) {
  if (w == 1) p[idx] = (uint8_t)v;
  else if (w == 2) reinterpret_cast<uint16_t*>(p)[idx] = (uint16_t)v;
  else reinterpret_cast<uint32_t*>(p)[idx] = v;
}

// Q[j][s] = R[j][s] - R[f][s], f = the first child of block j's parent (the
// block j - (jl mod tau), jl = j's index within its text's level): the parent
// and its first child start at the same position, so R[f] = R[parent].  Rows
// of a text's first level (no parent) are never read and are left as computed.
__global__ void k_relative_counts(const uint32_t* __restrict__ A, uint64_t c, uint32_t S,
                                  const uint32_t* __restrict__ text,
                                  const uint64_t* __restrict__ tfirst, uint32_t tau,
                                  uint8_t* __restrict__ q, uint32_t qw) {
  GRID_STRIDE(idx, c * S) {
    const uint64_t j = idx / S, sy = idx - j * S;
    const uint64_t jl = j - tfirst[text[j]];
    const uint64_t f = j - jl % tau;
    put_narrow(q, qw, idx, A[idx] - A[f * S + sy]);
  }
}

// Absolute rows of the texts that start at this level: entry e copies rows
// [src[e], src[e] + rows[e]) of A to [dst[e], ...) of out.
__global__ void k_root_rows(const uint32_t* __restrict__ A, uint32_t S,
                            const uint64_t* __restrict__ ent, uint32_t E,
                            uint32_t* __restrict__ out) {
  for (uint32_t e = blockIdx.x; e < E; e += gridDim.x) {
    const uint64_t src = ent[3 * e], rows = ent[3 * e + 1], dst = ent[3 * e + 2];
    for (uint64_t k = threadIdx.x; k < rows * S; k += blockDim.x) out[dst * S + k] = A[src * S + k];
  }
}

// msel[m] = index within its text's level of the m-th marked block of the
// level (m counted over the whole level; a text's marked blocks are contiguous).
__global__ void k_marked_index(const uint8_t* __restrict__ marked, const uint64_t* __restrict__ uoff,
                               uint64_t c, const uint32_t* __restrict__ text,
                               const uint64_t* __restrict__ tfirst, uint32_t* __restrict__ msel) {
  GRID_STRIDE(j, c) {
    if (marked[j]) msel[j - uoff[j]] = (uint32_t)(j - tfirst[text[j]]);
  }
}

// pcnt[u][s] for every unmarked block of a level (target t = tfirst + ptr_block).
__global__ __launch_bounds__(256) void k_pointer_counts(RankCtx rc, const uint64_t* st,
                                                        const uint32_t* text,
                                                        const uint8_t* marked, uint64_t c,
                                                        const uint64_t* uoff,
                                                        const uint64_t* tfirst,
                                                        const uint64_t* pb, const uint64_t* po,
                                                        const uint64_t* Rt, const uint32_t* cnt,
                                                        uint8_t* pcnt, uint32_t pw) {
  __shared__ uint32_t s_part[4][256];
  uint32_t* part = s_part[threadIdx.x >> 6];
  const int lane = lane_id();
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t j = gw; j < c; j += nw) {
    if (marked[j]) continue;  // wave-uniform
    const uint64_t u = uoff[j];
    const uint64_t tx = text[j];
    const uint64_t t = tfirst[tx] + pb[u];
    const uint64_t p = st[t] + po[u];
    wave_counts_before(rc, p, part);
    for (uint32_t s = lane; s < rc.S; s += 64)
      put_narrow(pcnt, pw, u * rc.S + s,
                 (uint32_t)(count_of(rc, p, part, s) - Rt[tx * rc.S + s] - cnt[t * rc.S + s]));
  }
}

// ---- launchers

hipError_t build_count_table(const uint8_t* T, uint64_t o0, uint64_t N, const int16_t* sym,
                             uint32_t S, uint32_t* H, uint64_t* B, uint64_t* G, hipStream_t s) {
  const uint64_t K = (N + kRankQ - 1) / kRankQ;
  const uint64_t nblk = (K + kColRows - 1) / kColRows;
  if (K) {
    k_chunk_hist<<<grid_for(K, 1, 16384), 256, 0, s>>>(T + o0, N, sym, S, K, H);
    k_col_block_sums<<<(unsigned)nblk, 256, 0, s>>>(H, K, S, B);
    k_col_block_scan<<<1, 256, 0, s>>>(B, nblk, S);
    k_col_scan<<<(unsigned)nblk, 256, 0, s>>>(H, K, S, B, G);
  } else {
    k_col_block_scan<<<1, 256, 0, s>>>(B, 0, S);  // no-op; G[0] is zeroed by the caller
  }
  return hipGetLastError();
}

hipError_t launch_text_rank_counts(const RankCtx& rc, const TextsDev& tx, uint64_t* Rt,
                                   uint64_t* Rtot, hipStream_t s) {
  k_text_counts<<<grid_for((uint64_t)tx.T * 64, 256, 1024), 256, 0, s>>>(rc, tx, Rt, Rtot);
  return hipGetLastError();
}

hipError_t launch_block_rank_counts(const RankCtx& rc, const uint64_t* st, const uint32_t* text,
                                    uint64_t c, const uint64_t* Rt, uint32_t* cnt, hipStream_t s) {
  if (!c) return hipSuccess;
  k_block_counts<<<grid_for(c * 64, 256, 4096), 256, 0, s>>>(rc, st, text, c, Rt, cnt);
  return hipGetLastError();
}

hipError_t launch_pointer_rank_counts(const RankCtx& rc, const uint64_t* st, const uint32_t* text,
                                      const uint8_t* marked, uint64_t c, const uint64_t* uoff,
                                      const uint64_t* tfirst, const uint64_t* pb,
                                      const uint64_t* po, const uint64_t* Rt, const uint32_t* cnt,
                                      uint8_t* pcnt, uint32_t pw, hipStream_t s) {
  if (!c) return hipSuccess;
  k_pointer_counts<<<grid_for(c * 64, 256, 4096), 256, 0, s>>>(rc, st, text, marked, c, uoff,
                                                                tfirst, pb, po, Rt, cnt, pcnt, pw);
  return hipGetLastError();
}

hipError_t launch_relative_counts(const uint32_t* A, uint64_t c, uint32_t S, const uint32_t* text,
                                  const uint64_t* tfirst, uint32_t tau, uint8_t* q, uint32_t qw,
                                  hipStream_t s) {
  if (!c) return hipSuccess;
  k_relative_counts<<<grid_for(c * S, 256), 256, 0, s>>>(A, c, S, text, tfirst, tau, q, qw);
  return hipGetLastError();
}

hipError_t launch_root_rows(const uint32_t* A, uint32_t S, const uint64_t* ent, uint32_t E,
                            uint32_t* out, hipStream_t s) {
  if (!E) return hipSuccess;
  k_root_rows<<<E < 4096 ? E : 4096, 256, 0, s>>>(A, S, ent, E, out);
  return hipGetLastError();
}

hipError_t launch_marked_index(const uint8_t* marked, const uint64_t* uoff, uint64_t c,
                               const uint32_t* text, const uint64_t* tfirst, uint32_t* msel,
                               hipStream_t s) {
  if (!c) return hipSuccess;
  k_marked_index<<<grid_for(c, 256), 256, 0, s>>>(marked, uoff, c, text, tfirst, msel);
  return hipGetLastError();
}

}  // namespace bt
