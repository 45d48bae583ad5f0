// Step (a2): prefix Karp-Rabin fingerprints over the whole text, computed once
// per build.  P[0] = 0, P[i+1] = P[i] * x + T[i] (mod 2^61 - 1); any window's
// fingerprint is then P[i+L] - P[i] * x^L (Section 2, phi with r = x).
//
// The recurrence is a prefix operation under the associative combine
// (h1, len1) o (h2, len2) = (h1 * x^len2 + h2, len1 + len2) (Section 2.2, the
// all-prefix operation).  One workgroup of 256 threads owns a 4096-byte tile:
//   1. each thread folds its 16 bytes by Horner's rule, as four independent
//      4-byte chains joined with x^4 (short dependency chains);
//   2. a wave64 shuffle scan and a 4-entry LDS pass give every thread the
//      fingerprint of the tile prefix before it;
//   3. the tile's carry-in comes from a decoupled look-back over the tile
//      status words (one 64-bit word per tile: value in bits 0..60, flag bits
//      61 (aggregate ready) and 62 (inclusive prefix ready));
//   4. each thread re-runs the four chains from its prefix and stages the 16
//      outputs in LDS so that the global stores are contiguous across the wave.
// Tile order comes from an atomic counter, so every tile a workgroup waits on
// was taken by a workgroup that started earlier.
#include "common.hpp"
#include "internal.hpp"

namespace bt {

constexpr uint64_t kFlagAgg = 1ull << 61;
constexpr uint64_t kFlagInc = 1ull << 62;

__global__ __launch_bounds__(kPfThreads) void k_prefix_fp(const uint8_t* __restrict__ T,
                                                          uint64_t n, uint64_t* __restrict__ P,
                                                          const PfPow* __restrict__ pw,
                                                          uint64_t* __restrict__ status,
                                                          uint32_t* __restrict__ ctr) {
  __shared__ uint64_t s_out[kPfThreads * 17];
  __shared__ uint64_t s_wave[kPfThreads / 64];
  __shared__ uint64_t s_excl;
  __shared__ uint32_t s_tile;

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = t >> 6;
  if (t == 0) s_tile = atomicAdd(ctr, 1u);
  __syncthreads();
  const uint64_t tile = s_tile;
  const uint64_t base = tile * kPfTile;
  const uint64_t pos = base + (uint64_t)t * kPfBytes;
  const uint64_t x = pw->x1[1];

  // 16 bytes per thread; zero beyond the end (those outputs are not stored).
  uint32_t w[4] = {0, 0, 0, 0};
  if (pos + kPfBytes <= n && ((reinterpret_cast<uintptr_t>(T) & 15) == 0)) {
    const uint4 v = *reinterpret_cast<const uint4*>(T + pos);
    w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
  } else {
    for (int k = 0; k < kPfBytes; ++k)
      if (pos + k < n) w[k >> 2] |= (uint32_t)T[pos + k] << (8 * (k & 3));
  }

  // 1. thread aggregate, as four independent 4-byte Horner chains combined by
  //    g_{c+1} = g_c * x^4 + h_c (short dependency chains keep the VALU busy)
  const auto byte_at = [&](int k) { return (uint64_t)((w[k >> 2] >> (8 * (k & 3))) & 0xFF); };
  uint64_t hc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    uint64_t v = byte_at(4 * c);
#pragma unroll
    for (int k = 1; k < 4; ++k) v = add61(mul61(v, x), byte_at(4 * c + k));
    hc[c] = v;
  }
  const uint64_t x4 = pw->x1[4];
  uint64_t g[4];
  g[0] = 0;
  g[1] = hc[0];
  g[2] = add61(mul61(g[1], x4), hc[1]);
  g[3] = add61(mul61(g[2], x4), hc[2]);
  const uint64_t h = add61(mul61(g[3], x4), hc[3]);

  // 2. wave inclusive scan: I = sum_{u <= lane} h_u x^(16 (lane - u))
  uint64_t I = h;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = __shfl_up(I, d);
    if (lane >= d) I = add61(mul61(o, pw->x16[d]), I);
  }
  uint64_t E = __shfl_up(I, 1);
  if (lane == 0) E = 0;
  if (lane == 63) s_wave[wv] = I;
  __syncthreads();
  uint64_t wp = 0, agg = 0;
#pragma unroll
  for (int v = 0; v < kPfThreads / 64; ++v) {
    if (v < wv) wp = add61(mul61(wp, pw->x16[64]), s_wave[v]);
    agg = add61(mul61(agg, pw->x16[64]), s_wave[v]);
  }
  const uint64_t local = add61(mul61(wp, pw->x16[lane]), E);

  // 3. carry-in from earlier tiles
  if (wv == 0) {
    uint64_t excl = 0;
    if (tile == 0) {
      if (lane == 0) st_relaxed(&status[0], kFlagInc | agg);
    } else {
      if (lane == 0) st_relaxed(&status[tile], kFlagAgg | agg);
      uint64_t mult = 1;
      int64_t look = (int64_t)tile - 1;
      while (true) {
        const int64_t pred = look - lane;
        uint64_t v = 0;
        if (pred >= 0) {
          do { v = ld_relaxed(&status[pred]); } while ((v >> 61) == 0);
        }
        const uint64_t inc = __ballot(pred >= 0 && (v & kFlagInc));
        const int stop = inc ? __ffsll((unsigned long long)inc) - 1 : 64;
        const uint64_t term = (lane <= stop && pred >= 0) ? mul61(v & kP61, pw->xt[lane]) : 0;
        excl = add61(excl, mul61(wave_sum61(term), mult));
        if (inc) break;
        mult = mul61(mult, pw->xt[64]);
        look -= 64;
      }
      if (lane == 0) st_relaxed(&status[tile], kFlagInc | add61(mul61(excl, pw->xt[1]), agg));
    }
    if (lane == 0) s_excl = excl;
  }
  __syncthreads();

  // 4. outputs P[pos+1 .. pos+16]: chain c restarts from C * x^(4c) + g_c
  const uint64_t C = add61(mul61(s_excl, pw->x16[t]), local);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    uint64_t v = c ? add61(mul61(C, pw->x1[4 * c]), g[c]) : C;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v = add61(mul61(v, x), byte_at(4 * c + k));
      s_out[t * 17 + 4 * c + k] = v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPfBytes; ++q) {
    const uint64_t m = (uint64_t)t + (uint64_t)kPfThreads * q;
    if (base + m < n) P[base + 1 + m] = s_out[(m >> 4) * 17 + (m & 15)];
  }
  if (tile == 0 && t == 0) P[0] = 0;
}

// The same tiled scan for the 32-bit pre-filter hash H[i+1] = H[i] * x32 + T[i]
// (mod 2^32, the wrap of uint32 arithmetic).  Tile status words hold the value
// in bits 0..31 and the flags in bits 32 (aggregate) and 33 (inclusive).
constexpr uint64_t kFlag32Agg = 1ull << 32;
constexpr uint64_t kFlag32Inc = 1ull << 33;

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  return v;
}

__global__ __launch_bounds__(kPfThreads) void k_prefix_h32(const uint8_t* __restrict__ T,
                                                           uint64_t n, uint32_t* __restrict__ H,
                                                           const PfPow32* __restrict__ pw,
                                                           uint64_t* __restrict__ status,
                                                           uint32_t* __restrict__ ctr) {
  __shared__ uint32_t s_out[kPfThreads * 17];
  __shared__ uint32_t s_wave[kPfThreads / 64];
  __shared__ uint32_t s_excl;
  __shared__ uint32_t s_tile;

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = t >> 6;
  if (t == 0) s_tile = atomicAdd(ctr, 1u);
  __syncthreads();
  const uint64_t tile = s_tile;
  const uint64_t base = tile * kPfTile;
  const uint64_t pos = base + (uint64_t)t * kPfBytes;
  const uint32_t x = pw->x1[1];

  uint32_t w[4] = {0, 0, 0, 0};
  if (pos + kPfBytes <= n && ((reinterpret_cast<uintptr_t>(T) & 15) == 0)) {
    const uint4 v = *reinterpret_cast<const uint4*>(T + pos);
    w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
  } else {
    for (int k = 0; k < kPfBytes; ++k)
      if (pos + k < n) w[k >> 2] |= (uint32_t)T[pos + k] << (8 * (k & 3));
  }
  const auto byte_at = [&](int k) { return (w[k >> 2] >> (8 * (k & 3))) & 0xFFu; };

  // thread aggregate: four 4-byte Horner chains joined with x^4
  uint32_t hc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    uint32_t v = byte_at(4 * c);
#pragma unroll
    for (int k = 1; k < 4; ++k) v = v * x + byte_at(4 * c + k);
    hc[c] = v;
  }
  const uint32_t x4 = pw->x1[4];
  uint32_t g[4];
  g[0] = 0;
  g[1] = hc[0];
  g[2] = g[1] * x4 + hc[1];
  g[3] = g[2] * x4 + hc[2];
  const uint32_t h = g[3] * x4 + hc[3];

  uint32_t I = h;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(I, d);
    if (lane >= d) I = o * pw->x16[d] + I;
  }
  uint32_t E = __shfl_up(I, 1);
  if (lane == 0) E = 0;
  if (lane == 63) s_wave[wv] = I;
  __syncthreads();
  uint32_t wp = 0, agg = 0;
#pragma unroll
  for (int v = 0; v < kPfThreads / 64; ++v) {
    if (v < wv) wp = wp * pw->x16[64] + s_wave[v];
    agg = agg * pw->x16[64] + s_wave[v];
  }
  const uint32_t local = wp * pw->x16[lane] + E;

  if (wv == 0) {
    uint32_t excl = 0;
    if (tile == 0) {
      if (lane == 0) st_relaxed(&status[0], kFlag32Inc | agg);
    } else {
      if (lane == 0) st_relaxed(&status[tile], kFlag32Agg | agg);
      uint32_t mult = 1;
      int64_t look = (int64_t)tile - 1;
      while (true) {
        const int64_t pred = look - lane;
        uint64_t v = 0;
        if (pred >= 0) {
          do { v = ld_relaxed(&status[pred]); } while ((v >> 32) == 0);
        }
        const uint64_t inc = __ballot(pred >= 0 && (v & kFlag32Inc));
        const int stop = inc ? __ffsll((unsigned long long)inc) - 1 : 64;
        const uint32_t term = (lane <= stop && pred >= 0) ? (uint32_t)v * pw->xt[lane] : 0u;
        excl += wave_sum32(term) * mult;
        if (inc) break;
        mult *= pw->xt[64];
        look -= 64;
      }
      if (lane == 0) st_relaxed(&status[tile], kFlag32Inc | (uint32_t)(excl * pw->xt[1] + agg));
    }
    if (lane == 0) s_excl = excl;
  }
  __syncthreads();

  const uint32_t C = s_excl * pw->x16[t] + local;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    uint32_t v = c ? C * pw->x1[4 * c] + g[c] : C;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v = v * x + byte_at(4 * c + k);
      s_out[t * 17 + 4 * c + k] = v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPfBytes; ++q) {
    const uint64_t m = (uint64_t)t + (uint64_t)kPfThreads * q;
    if (base + m < n) H[base + 1 + m] = s_out[(m >> 4) * 17 + (m & 15)];
  }
  if (tile == 0 && t == 0) H[0] = 0;
}

__global__ void k_zero_u32(uint32_t* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void k_zero_u64(uint64_t* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

hipError_t launch_prefix_fp(const uint8_t* T, uint64_t n, uint64_t* P, const PfPow* pw,
                            uint64_t* status, uint32_t* ctr, hipStream_t s) {
  const uint64_t tiles = (n + kPfTile - 1) / kPfTile;
  if (tiles == 0) {
    // P[0] = 0 only
    k_zero_u64<<<1, 64, 0, s>>>(P, 1);
    return hipGetLastError();
  }
  // status words and the tile counter (adjacent: ctr is the word after status)
  const uint64_t zn = tiles + 1;
  const unsigned zb = (unsigned)((zn + 255) / 256 < 4096 ? (zn + 255) / 256 : 4096);
  k_zero_u64<<<zb, 256, 0, s>>>(status, tiles);
  k_zero_u64<<<1, 64, 0, s>>>(reinterpret_cast<uint64_t*>(ctr), 1);
  k_prefix_fp<<<(unsigned)tiles, kPfThreads, 0, s>>>(T, n, P, pw, status, ctr);
  return hipGetLastError();
}

hipError_t launch_prefix_h32(const uint8_t* T, uint64_t n, uint32_t* H, const PfPow32* pw,
                             uint64_t* status, uint32_t* ctr, hipStream_t s) {
  const uint64_t tiles = (n + kPfTile - 1) / kPfTile;
  if (tiles == 0) {
    // H[0] = 0 only
    k_zero_u32<<<1, 64, 0, s>>>(H, 1);
    return hipGetLastError();
  }
  const uint64_t zn = tiles + 1;
  const unsigned zb = (unsigned)((zn + 255) / 256 < 4096 ? (zn + 255) / 256 : 4096);
  k_zero_u64<<<zb, 256, 0, s>>>(status, tiles);
  k_zero_u64<<<1, 64, 0, s>>>(reinterpret_cast<uint64_t*>(ctr), 1);
  k_prefix_h32<<<(unsigned)tiles, kPfThreads, 0, s>>>(T, n, H, pw, status, ctr);
  return hipGetLastError();
}

}  // namespace bt
