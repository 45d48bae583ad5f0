// Fills and a device-wide exclusive prefix sum (Section 2.2, prefix sums) used
// by the compaction steps of every level.  Reduce-then-scan over 2048-element
// tiles; the tile sums are scanned recursively.
#include "common.hpp"
#include "internal.hpp"

namespace bt {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr uint64_t kScanTile = kScanThreads * kScanItems;

template <typename Tp>
__global__ void k_fill(Tp* p, Tp v, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

static unsigned grid_for(uint64_t n, unsigned threads, unsigned cap = 8192) {
  uint64_t g = (n + threads - 1) / threads;
  if (g == 0) g = 1;
  return (unsigned)(g < cap ? g : cap);
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  k_fill<uint64_t><<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  k_fill<uint32_t><<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, uint64_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  k_fill<uint8_t><<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

// Several fills in one launch: job y = blockIdx.y fills words[y] 32-bit words
// at p[y] with value[y], 16 bytes per store where the buffer allows.
__global__ void k_fill_many(FillList f) {
  const int y = blockIdx.y;
  uint32_t* p = f.p[y];
  const uint64_t n = f.words[y];
  const uint32_t v = f.value[y];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t head = ((reinterpret_cast<uintptr_t>(p) & 15) == 0) ? 0 : n;  // unaligned: scalar only
  const uint64_t nq = (n - head) / 4;
  uint4* q = reinterpret_cast<uint4*>(p);
  const uint4 vv = make_uint4(v, v, v, v);
  for (uint64_t i = tid; i < nq; i += stride) q[i] = vv;
  for (uint64_t i = 4 * nq + tid; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_many(const FillList& f, hipStream_t s) {
  uint64_t most = 0;
  for (int k = 0; k < f.n; ++k) most = f.words[k] > most ? f.words[k] : most;
  if (!f.n || !most) return hipSuccess;
  const dim3 grid(grid_for((most + 3) / 4, 256, 4096), (unsigned)f.n);
  k_fill_many<<<grid, 256, 0, s>>>(f);
  return hipGetLastError();
}

// Exclusive scan of one block's values (256 threads); returns the block total.
__device__ uint64_t block_excl_scan(uint64_t v, uint64_t* s_w) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint64_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = __shfl_up(inc, d);
    if (lane >= d) inc += o;
  }
  if (lane == 63) s_w[wv] = inc;
  __syncthreads();
  uint64_t before = 0, total = 0;
#pragma unroll
  for (int k = 0; k < kScanThreads / 64; ++k) {
    if (k < wv) before += s_w[k];
    total += s_w[k];
  }
  __syncthreads();
  return before + inc - v + 0 * total;
}

__device__ uint64_t block_total(uint64_t v, uint64_t* s_w) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  if (lane == 0) s_w[wv] = v;
  __syncthreads();
  uint64_t total = 0;
#pragma unroll
  for (int k = 0; k < kScanThreads / 64; ++k) total += s_w[k];
  __syncthreads();
  return total;
}

// Tile sums.
__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const uint64_t* __restrict__ a,
                                                            uint64_t n, uint64_t* sums) {
  __shared__ uint64_t s_w[kScanThreads / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint64_t v = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = base + (uint64_t)k * kScanThreads + threadIdx.x;
    if (i < n) v += a[i];
  }
  const uint64_t tot = block_total(v, s_w);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Scan each tile in place and add its carry-in (carry == nullptr: none); the
// thread holding element n-1 (or the first thread when n == 0) also stores the
// grand total in a[n].  Wave w of the tile owns its elements 512 w .. 512 w +
// 511 as eight rows of 64 (lane l: element 64 k + l of row k), so every load
// and store is one contiguous 512-byte run; each row is scanned with shuffles
// and the rows are chained, then the waves' totals give their offsets.
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(uint64_t* __restrict__ a, uint64_t n,
                                                            const uint64_t* __restrict__ carry) {
  __shared__ uint64_t s_w[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t wbase = (uint64_t)blockIdx.x * kScanTile + (uint64_t)wv * (64 * kScanItems);
  uint64_t v[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = wbase + 64ull * k + lane;
    v[k] = i < n ? a[i] : 0;
  }
  // v[k] becomes the wave's exclusive prefix at its element; the element n-1
  // keeps its inclusive prefix for a[n]
  uint64_t run = 0, incl_last = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t orig = v[k];
    uint64_t x = orig;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t o = __shfl_up(x, d);
      if (lane >= d) x += o;
    }
    v[k] = run + x - orig;
    if (n && wbase + 64ull * k + lane == n - 1) incl_last = run + x;
    run += __shfl(x, 63);
  }
  if (lane == 0) s_w[wv] = run;
  __syncthreads();
  uint64_t off = carry ? carry[blockIdx.x] : 0;
#pragma unroll
  for (int k = 0; k < kScanThreads / 64; ++k)
    if (k < wv) off += s_w[k];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t i = wbase + 64ull * k + lane;
    if (i < n) a[i] = off + v[k];
  }
  if (n == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) a[0] = off;
  } else if (n - 1 >= wbase && n - 1 < wbase + 64ull * kScanItems &&
             lane == (int)((n - 1 - wbase) & 63)) {
    a[n] = off + incl_last;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_text_step(uint32_t T, const uint64_t* __restrict__ cs,
                                                            const uint64_t* __restrict__ tfirst,
                                                            const uint64_t* __restrict__ tcount,
                                                            const uint64_t* __restrict__ enter,
                                                            const uint64_t* __restrict__ uoff,
                                                            uint64_t* __restrict__ ncount,
                                                            uint64_t* __restrict__ nfirst,
                                                            uint64_t* __restrict__ tu) {
  __shared__ uint64_t s_w[kScanThreads / 64];
  const uint64_t first = (uint64_t)threadIdx.x * kScanItems;
  uint64_t v[kScanItems];
  uint64_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t t = first + k;
    v[k] = 0;
    if (t < T) {
      const uint64_t f = tfirst[t], e = f + tcount[t];
      v[k] = cs[e] - cs[f] + enter[t];
      ncount[t] = v[k];
      tu[t] = uoff[e] - uoff[f];
    }
    sum += v[k];
  }
  uint64_t run = block_excl_scan(sum, s_w);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t t = first + k;
    if (t < T) nfirst[t] = run;
    run += v[k];
    if (t + 1 == T || (T == 0 && t == 0)) nfirst[T] = run;
  }
}

hipError_t launch_text_step(uint32_t T, const uint64_t* cs, const uint64_t* tfirst,
                            const uint64_t* tcount, const uint64_t* enter, const uint64_t* uoff,
                            uint64_t* ncount, uint64_t* nfirst, uint64_t* tu, hipStream_t s) {
  if (T > kTextStepMax) return hipErrorInvalidValue;
  static_assert(kTextStepMax == kScanTile, "one workgroup scans the texts");
  k_text_step<<<1, kScanThreads, 0, s>>>(T, cs, tfirst, tcount, enter, uoff, ncount, nfirst, tu);
  return hipGetLastError();
}

uint64_t scan_tmp_words(uint64_t n) {
  uint64_t w = 0;
  while (n > kScanTile) {
    const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
    w += tiles + 1;
    n = tiles;
  }
  return w + 1;
}

hipError_t scan_excl_u64(uint64_t* a, uint64_t n, uint64_t* tmp, hipStream_t s) {
  if (n <= kScanTile) {
    k_tile_scan<<<1, kScanThreads, 0, s>>>(a, n, nullptr);
    return hipGetLastError();
  }
  const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
  uint64_t* sums = tmp;
  k_tile_sums<<<(unsigned)tiles, kScanThreads, 0, s>>>(a, n, sums);
  hipError_t e = scan_excl_u64(sums, tiles, tmp + tiles + 1, s);
  if (e != hipSuccess) return e;
  k_tile_scan<<<(unsigned)tiles, kScanThreads, 0, s>>>(a, n, sums);
  return hipGetLastError();
}

}  // namespace bt
