// Step (a2): prefix Karp-Rabin fingerprints over the whole text, computed once
// per build.  P[0] = 0, P[i+1] = P[i] * x + T[i] (mod 2^61 - 1); any window's
// fingerprint is then P[i+L] - P[i] * x^L (Section 2, phi with r = x).  The
// same pass computes, in arithmetic mod 2^32 with another (odd) base, the
// 32-bit pre-filter hashes H of the probe scan.
//
// The recurrence is a prefix operation under the associative combine
// (h1, len1) o (h2, len2) = (h1 * x^len2 + h2, len1 + len2) (Section 2.2, the
// all-prefix operation).  Workgroups of 512 threads stay resident and take
// 32 KiB tiles in order from an atomic counter; in a tile each thread owns 64
// consecutive bytes.
//   1. Fold: the thread's bytes in groups of eight; a group's fingerprint
//      sum_k b_k x^(7-k) is seven lookups in LDS tables of b x^j plus one
//      reduction (no multiplication mod 2^61 - 1 per byte), its 32-bit hash
//      eight multiply-adds; the eight groups join with x^8.
//   2. A wave64 shuffle scan and a 4-entry LDS pass give each thread the fold
//      of the tile before it, and the tile aggregate.
//   3. The tile's carry-in comes from a decoupled look-back over the tile
//      status words (value plus two flag bits: aggregate ready, inclusive
//      prefix ready); wave 0 runs it for the fingerprints and wave 1 for the
//      32-bit hashes, side by side.
//   4. Outputs: every 16th value (the thread's prefix times x^(16 c) plus the
//      folds of step 1) goes to LDS; then, row by row (16 bytes per thread), each
//      thread runs 16 Horner steps from one of them (one multiply-add per
//      output), and each wave stages its outputs in LDS so that its stores are
//      lane-contiguous.  The sampled form stores every 16th value only:
//      P[16 q] for 16 q <= n (and, with sampled hashes, H[16 q] likewise).
// Tile order comes from the counter, so a tile waits only on tiles that
// running workgroups hold.  The text is read once for both results.
#include "common.hpp"
#include "internal.hpp"

namespace bt {
namespace {

constexpr unsigned kPfGrid = 1024;  // resident workgroups
constexpr uint64_t kPfRow = (uint64_t)kPfThreads * 16;  // step-4 row: 16 bytes per thread

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// s mod (2^61 - 1) for any 64-bit s.
__device__ __forceinline__ uint64_t fold61(uint64_t s) {
  s = (s & kP61) + (s >> 61);
  return s >= kP61 ? s - kP61 : s;
}

struct A61 {
  using V = uint64_t;
  static constexpr uint64_t kAgg = 1ull << 61;  // status flags above the value
  static constexpr uint64_t kInc = 1ull << 62;
  __device__ static V mul(V a, V b) { return mad61(a, b, 0); }
  __device__ static V add(V a, V b) { return add61(a, b); }
  __device__ static V value(uint64_t w) { return w & kP61; }
  __device__ static bool ready(uint64_t w) { return (w >> 61) != 0; }
  __device__ static V wave_sum(V v) { return wave_sum61(v); }
};

struct A32 {
  using V = uint32_t;
  static constexpr uint64_t kAgg = 1ull << 32;
  static constexpr uint64_t kInc = 1ull << 33;
  __device__ static V mul(V a, V b) { return a * b; }
  __device__ static V add(V a, V b) { return a + b; }
  __device__ static V value(uint64_t w) { return (uint32_t)w; }
  __device__ static bool ready(uint64_t w) { return (w >> 32) != 0; }
  __device__ static V wave_sum(V v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
  }
};

// One wave: publish the tile aggregate, fold the predecessors' values (64 at a
// time, stopping at the first inclusive prefix), publish the inclusive prefix.
// Returns the fold of everything before the tile (all lanes).  xt[k] is the
// power for k tiles.
template <class A>
__device__ typename A::V look_back(uint64_t* status, uint64_t tile, typename A::V agg,
                                   const typename A::V* __restrict__ xt) {
  using V = typename A::V;
  const int lane = lane_id();
  if (tile == 0) {
    if (lane == 0) st_relaxed(&status[0], A::kInc | (uint64_t)agg);
    return 0;
  }
  if (lane == 0) st_relaxed(&status[tile], A::kAgg | (uint64_t)agg);
  const V xl = xt[lane], x64 = xt[64];
  V excl = 0, mult = 1;
  int64_t look = (int64_t)tile - 1;
  while (true) {
    const int64_t pred = look - lane;
    uint64_t v = 0;
    if (pred >= 0) {
      do { v = ld_relaxed(&status[pred]); } while (!A::ready(v));
    }
    const uint64_t inc = __ballot(pred >= 0 && (v & A::kInc));
    const int stop = inc ? __ffsll((unsigned long long)inc) - 1 : 64;
    const V term = (lane <= stop && pred >= 0) ? A::mul(A::value(v), xl) : (V)0;
    excl = A::add(excl, A::mul(A::wave_sum(term), mult));
    if (inc) break;
    mult = A::mul(mult, x64);
    look -= 64;
  }
  if (lane == 0) st_relaxed(&status[tile], A::kInc | (uint64_t)A::add(A::mul(excl, xt[1]), agg));
  return excl;
}

// Two waves per SIMD: the register budget of three spilled, and ran slower.
// Q4 (not SAMPLED): the fingerprints every 4th position, Ps[q] = P[4 q].
template <bool SAMPLED, bool WH, bool HS, bool Q4>
__global__ __launch_bounds__(kPfThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_prefix(
    const uint8_t* __restrict__ T, uint64_t n, uint64_t* __restrict__ P, uint32_t* __restrict__ H,
    const PfTab* __restrict__ tb, uint64_t* __restrict__ st61, uint64_t* __restrict__ st32,
    uint32_t* __restrict__ ctr, uint64_t tiles) {
  __shared__ uint64_t s_g61[7 * 256];
  __shared__ uint64_t s_w61[kPfThreads / 64];
  __shared__ uint32_t s_w32[kPfThreads / 64];
  __shared__ uint64_t s_ex61;
  __shared__ uint32_t s_ex32;
  __shared__ uint32_t s_tile;
  // chain starts P[16 m], H[16 m] of the tile (m = 0..1023), and per wave a
  // staging area: 64 rows of 8 fingerprints, or of 16 hashes (row strides 9
  // and 17 words keep the lanes on different banks)
  constexpr bool DENSE = !SAMPLED && !Q4;
  __shared__ uint64_t s_st61[DENSE ? kPfTile / 16 : 1];
  __shared__ uint32_t s_st32[(WH && !HS) ? kPfTile / 16 : 1];
  __shared__ uint64_t s_out[(DENSE || (WH && !HS)) ? (kPfThreads / 64) * 64 * 9 : 1];

  const int t0 = threadIdx.x;
  for (int k = t0; k < 7 * 256; k += kPfThreads) s_g61[k] = (&tb->g61[0][0])[k];
  const uint64_t x1 = tb->x1_61, x8 = tb->x8_61;
  const uint32_t y1 = tb->x1_32, y8 = tb->x8_32;
  const bool t_al = (reinterpret_cast<uintptr_t>(T) & 15) == 0;

  while (true) {
    // The thread index is hidden from the optimizer in every pass: otherwise
    // the addresses derived from it are hoisted out of the tile loop and held
    // in registers for its whole length.
    int t = t0;
    asm volatile("" : "+v"(t));
    const int lane = t & 63;
    const int wv = t >> 6;
    if (t == 0) s_tile = atomicAdd(ctr, 1u);
    __syncthreads();  // (first pass: the tables are in LDS too)
    const uint64_t tile = s_tile;
    if (tile >= tiles) break;
    const uint64_t pos = tile * kPfTile + (uint64_t)t * kPfBytes;
    const bool full = pos + kPfBytes <= n;

    // the thread's 64 bytes, zero past the end (no stored value depends on
    // them, and only the last tile, whose aggregate nobody reads, has any)
    uint32_t w[16];
    if (t_al && full) {
      const uint4* src = reinterpret_cast<const uint4*>(T + pos);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint4 v = src[q];
        w[4 * q] = v.x;
        w[4 * q + 1] = v.y;
        w[4 * q + 2] = v.z;
        w[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) w[k] = 0;
#pragma unroll
      for (int k = 0; k < kPfBytes; ++k)
        if (pos + k < n) w[k >> 2] |= (uint32_t)T[pos + k] << (8 * (k & 3));
    }
    const auto byte_at = [&](int k) { return (w[k >> 2] >> (8 * (k & 3))) & 0xFFu; };

    // 1. folds: h = all 64 bytes; F[c] = the first 16 c bytes (c = 1..3)
    uint64_t h61 = 0, F61[4] = {0, 0, 0, 0};
    uint32_t h32 = 0, F32[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      uint64_t g = byte_at(8 * q + 7);
#pragma unroll
      for (int j = 1; j < 8; ++j)
        g += s_g61[(j - 1) * 256 + byte_at(8 * q + 7 - j)];  // eight terms below 2^61
      // the 32-bit hash by Horner's rule: a 32-bit multiply-add per byte is
      // cheaper than a lookup in the one LDS pipe the workgroup shares
      uint32_t g32 = 0;
      if (WH) {
#pragma unroll
        for (int k = 0; k < 8; ++k) g32 = g32 * y1 + byte_at(8 * q + k);
      }
      g = fold61(g);
      h61 = q ? mad61(h61, x8, g) : g;
      if (WH) h32 = q ? h32 * y8 + g32 : g32;
      if ((q & 1) && q < 7) {
        F61[(q + 1) >> 1] = h61;
        F32[(q + 1) >> 1] = h32;
      }
      // one group's lookups in flight at a time (registers)
      __builtin_amdgcn_sched_barrier(0);
    }

    // 16 bytes of a row of step 4 (row r: tile offset kPfRow r + 16 t)
    const uint64_t tb0 = tile * kPfTile;
    const auto load_row = [&](int r, uint32_t* bw) {
      const uint64_t q = tb0 + kPfRow * r + 16 * (uint64_t)t;
#pragma unroll
      for (int e = 0; e < 4; ++e) bw[e] = 0;
      if (t_al && q + 16 <= n) {
        const uint4 x = *reinterpret_cast<const uint4*>(T + q);
        bw[0] = x.x;
        bw[1] = x.y;
        bw[2] = x.z;
        bw[3] = x.w;
      } else {
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (q + k < n) bw[k >> 2] |= (uint32_t)T[q + k] << (8 * (k & 3));
      }
    };
    // row 0 is requested now: the scan and the look-back hide its latency
    uint32_t rw[4];
    if (DENSE || WH) load_row(0, rw);

    // 2. inclusive wave scan with x^(64 d); the exclusive value, the wave
    //    aggregates, the fold of the earlier waves and the tile aggregate
    uint64_t I = h61;
    uint32_t I32 = h32;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t o = __shfl_up(I, d);
      const uint32_t o32 = WH ? __shfl_up(I32, d) : 0u;
      if (lane >= d) {
        I = mad61(o, tb->t61[d], I);
        if (WH) I32 = o32 * tb->t32[d] + I32;
      }
    }
    uint64_t E = __shfl_up(I, 1);
    uint32_t E32 = WH ? __shfl_up(I32, 1) : 0u;
    if (lane == 0) {
      E = 0;
      E32 = 0;
    }
    if (lane == 63) {
      s_w61[wv] = I;
      if (WH) s_w32[wv] = I32;
    }
    __syncthreads();
    uint64_t wp = 0, agg = 0;
    uint32_t wp32 = 0, agg32 = 0;
    const uint64_t xw = tb->t61[64];
    const uint32_t yw = tb->t32[64];
#pragma unroll
    for (int v = 0; v < kPfThreads / 64; ++v) {
      const uint64_t a = s_w61[v];
      if (v < wv) wp = mad61(wp, xw, a);
      agg = mad61(agg, xw, a);
      if (WH) {
        const uint32_t a32 = s_w32[v];
        if (v < wv) wp32 = wp32 * yw + a32;
        agg32 = agg32 * yw + a32;
      }
    }
    const uint64_t local = mad61(wp, tb->t61[lane], E);  // tile bytes before this thread
    const uint32_t local32 = wp32 * tb->t32[lane] + E32;

    // 3. carry-in
    if (wv == 0) {
      const uint64_t ex = look_back<A61>(st61, tile, agg, tb->xt61);
      if (lane == 0) s_ex61 = ex;
    }
    if (WH && wv == 1) {
      const uint32_t ex = look_back<A32>(st32, tile, agg32, tb->xt32);
      if (lane == 0) s_ex32 = ex;
    }
    __syncthreads();
    const uint64_t C = mad61(s_ex61, tb->t61[t], local);  // P[pos]
    const uint32_t C32 = s_ex32 * tb->t32[t] + local32;  // H[pos]

    // 4. chain starts, then outputs.  Thread t of the contiguous layout holds
    // P[pos + 16 c] = C x^(16 c) + F[c].  The outputs are written in rows of
    // 16 bytes per thread: in row r thread t runs the 16 Horner steps from tile offset
    // kPfRow r + 16 t, and each wave stages its 64 chains in LDS so that every
    // store instruction covers whole 64-byte runs (lane-contiguous).
    {
      uint64_t v[4];
      uint32_t u[4];
      v[0] = C;
      u[0] = C32;
#pragma unroll
      for (int c = 1; c < 4; ++c) {
        v[c] = mad61(C, tb->c61[c], F61[c]);
        u[c] = C32 * tb->c32[c] + F32[c];
      }
      if (SAMPLED) {
        if (pos <= n) {
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (pos + 16 * c <= n) P[(pos >> 4) + c] = v[c];
          if (pos + kPfBytes == n) P[n >> 4] = mad61(C, tb->t61[1], h61);
        }
      } else if (Q4) {
        // every 4th: from each P[pos + 16 c], four Horner steps at a time
        if (pos <= n) {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            uint64_t val = v[c];
#pragma unroll
            for (int d = 0; d < 4; ++d) {
              const uint64_t q = pos + 16 * c + 4 * d;
              if (q <= n) P[q >> 2] = val;
              if (d < 3) {
#pragma unroll
                for (int e = 0; e < 4; ++e) val = mad61(val, x1, byte_at(16 * c + 4 * d + e));
              }
            }
          }
          if (pos + kPfBytes == n) P[n >> 2] = mad61(C, tb->t61[1], h61);
        }
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) s_st61[4 * t + c] = v[c];
      }
      if (HS) {
        if (pos <= n) {
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (pos + 16 * c <= n) H[(pos >> 4) + c] = u[c];
          if (pos + kPfBytes == n) H[n >> 4] = C32 * tb->t32[1] + h32;
        }
      } else if (WH) {
#pragma unroll
        for (int c = 0; c < 4; ++c) s_st32[4 * t + c] = u[c];
      }
    }
    if (DENSE || (WH && !HS)) {
      __syncthreads();
      const bool tfull = tb0 + kPfTile < n;  // no output of the tile lies past n
      uint64_t* so = s_out + wv * 64 * 9;
      uint32_t* so32 = reinterpret_cast<uint32_t*>(so);
#pragma unroll 1
      for (int r = 0; r < 4; ++r) {
        const uint64_t q = tb0 + kPfRow * r + 16 * (uint64_t)t;  // this thread's 16 bytes
        const uint64_t wbase = tb0 + kPfRow * r + 1024 * (uint64_t)wv;  // the wave's 1024
        uint32_t nx[4];  // the next row's bytes, requested one row ahead
        if (r < 3) load_row(r + 1, nx);
        const auto rb = [&](int k) { return (rw[k >> 2] >> (8 * (k & 3))) & 0xFFu; };
        if (DENSE) {
          // two halves of eight steps: P[q + 8 h + k] to row `lane`, then the
          // wave stores 512 values, runs of eight (64 bytes) per lane group
          uint64_t val = s_st61[kPfThreads * r + t];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              so[lane * 9 + k] = val;
              val = mad61(val, x1, rb(8 * h + k));
            }
            wave_sync();
#pragma unroll
            for (int m = 0; m < 8; ++m) {
              const int e = 64 * m + lane;  // row e / 8, step e % 8
              const uint64_t j = wbase + 16 * (uint64_t)(e >> 3) + 8 * h + (e & 7);
              if (tfull || j <= n) P[j] = so[(e >> 3) * 9 + (e & 7)];
            }
            wave_sync();
          }
          if (q + 16 == n) P[n] = val;
        }
        if (WH && !HS) {
          uint32_t val = s_st32[kPfThreads * r + t];
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            so32[lane * 17 + k] = val;
            val = val * y1 + rb(k);
          }
          wave_sync();
#pragma unroll
          for (int m = 0; m < 16; ++m) {
            const int e = 64 * m + lane;
            const uint64_t j = wbase + e;
            if (tfull || j <= n) H[j] = so32[(e >> 4) * 17 + (e & 15)];
          }
          wave_sync();
          if (q + 16 == n) H[n] = val;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) rw[e] = nx[e];
      }
    }
    __syncthreads();  // s_tile, s_w*, s_ex* are rewritten by the next tile
  }
}

template <typename V>
__global__ void k_zero(V* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

}  // namespace

hipError_t launch_prefix(const uint8_t* T, uint64_t n, uint64_t* P, bool sampled, uint32_t* H,
                         const PfTab* tab, uint64_t* status, hipStream_t s, bool hsampled,
                         bool quarter) {
  const uint64_t tiles = (n + kPfTile - 1) / kPfTile;
  if (tiles == 0) {  // P[0] = 0 (and H[0] = 0) only
    k_zero<uint64_t><<<1, 64, 0, s>>>(P, 1);
    if (H) k_zero<uint32_t><<<1, 64, 0, s>>>(H, 1);
    return hipGetLastError();
  }
  const uint64_t words = prefix_status_words(n);
  const unsigned zb = (unsigned)((words + 255) / 256 < 4096 ? (words + 255) / 256 : 4096);
  k_zero<uint64_t><<<zb, 256, 0, s>>>(status, words);
  uint64_t* st61 = status;
  uint64_t* st32 = status + tiles + 1;
  uint32_t* ctr = reinterpret_cast<uint32_t*>(status + 2 * (tiles + 1));
  const unsigned grid = (unsigned)(tiles < kPfGrid ? tiles : kPfGrid);
  if (quarter && (sampled || hsampled || !H)) return hipErrorInvalidValue;
  if (sampled && hsampled) {
    if (!H) return hipErrorInvalidValue;
    k_prefix<true, true, true, false><<<grid, kPfThreads, 0, s>>>(T, n, P, H, tab, st61, st32, ctr, tiles);
  } else if (sampled) {
    if (H) k_prefix<true, true, false, false><<<grid, kPfThreads, 0, s>>>(T, n, P, H, tab, st61, st32, ctr, tiles);
    else k_prefix<true, false, false, false><<<grid, kPfThreads, 0, s>>>(T, n, P, H, tab, st61, st32, ctr, tiles);
  } else if (quarter) {
    k_prefix<false, true, false, true><<<grid, kPfThreads, 0, s>>>(T, n, P, H, tab, st61, st32, ctr, tiles);
  } else {
    if (hsampled) return hipErrorInvalidValue;
    if (H) k_prefix<false, true, false, false><<<grid, kPfThreads, 0, s>>>(T, n, P, H, tab, st61, st32, ctr, tiles);
    else k_prefix<false, false, false, false><<<grid, kPfThreads, 0, s>>>(T, n, P, H, tab, st61, st32, ctr, tiles);
  }
  return hipGetLastError();
}

}  // namespace bt
