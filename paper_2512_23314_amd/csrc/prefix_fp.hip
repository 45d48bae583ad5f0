// Step (a2): prefix Karp-Rabin fingerprints over the whole text, computed once
// per build.  P[0] = 0, P[i+1] = P[i] * x + T[i] (mod 2^61 - 1); any window's
// fingerprint is then P[i+L] - P[i] * x^L (Section 2, phi with r = x).  The
// same scan, in arithmetic mod 2^32 with another (odd) base, gives the 32-bit
// pre-filter hashes H of the probe scan.
//
// The recurrence is a prefix operation under the associative combine
// (h1, len1) o (h2, len2) = (h1 * x^len2 + h2, len1 + len2) (Section 2.2, the
// all-prefix operation).  One workgroup of 256 threads owns a 16 KiB tile of
// four 4 KiB rows; in each row a thread owns 16 consecutive bytes:
//   1. each thread folds its 16 bytes of every row by Horner's rule, as four
//      independent 4-byte chains joined with x^4 (short dependency chains);
//   2. per row, a wave64 shuffle scan and a 4-entry LDS pass give every thread
//      the fingerprint of the row prefix before it; the row aggregates fold
//      into the tile aggregate;
//   3. the tile's carry-in comes from a decoupled look-back over the tile
//      status words (value plus two flag bits: aggregate ready, inclusive
//      prefix ready);
//   4. row by row, each thread re-runs its four chains from its prefix and
//      stages the 16 outputs in LDS so that the global stores are contiguous.
// Tile order comes from an atomic counter, so every tile a workgroup waits on
// was taken by a workgroup that started earlier.  The sampled form (SAMPLED)
// stores every 16th value only, P[16 q] for 16 q <= n: each thread's value
// before its 16 bytes, plus P[n] when n is a multiple of 16; any other value is
// 15 Horner steps or fewer from its sample.  Returning atomics on one
// address serialize (about 10 ns apart), which is why a tile spans four rows:
// one counter update per 16 KiB.
#include "common.hpp"
#include "internal.hpp"

namespace bt {

// Arithmetic of the two scans.
struct Mod61 {
  using V = uint64_t;
  using Pow = PfPow;
  static constexpr uint64_t kAgg = 1ull << 61;  // status flags above the value
  static constexpr uint64_t kInc = 1ull << 62;
  __device__ static V mul(V a, V b) { return mul61(a, b); }
  __device__ static V add(V a, V b) { return add61(a, b); }
  __device__ static V value(uint64_t w) { return w & kP61; }
  __device__ static bool ready(uint64_t w) { return (w >> 61) != 0; }
  __device__ static V wave_sum(V v) { return wave_sum61(v); }
};

struct Mod32 {
  using V = uint32_t;
  using Pow = PfPow32;
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

template <class A, bool SAMPLED>
__global__ __launch_bounds__(kPfThreads) void k_prefix(const uint8_t* __restrict__ T, uint64_t n,
                                                       typename A::V* __restrict__ P,
                                                       const typename A::Pow* __restrict__ pw,
                                                       uint64_t* __restrict__ status,
                                                       uint32_t* __restrict__ ctr) {
  using V = typename A::V;
  __shared__ V s_out[kPfThreads * 17];
  __shared__ V s_wave[kPfRows][kPfThreads / 64];
  __shared__ V s_excl;
  __shared__ uint32_t s_tile;

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = t >> 6;
  if (t == 0) s_tile = atomicAdd(ctr, 1u);
  __syncthreads();
  const uint64_t tile = s_tile;
  const uint64_t base = tile * kPfTile;
  const V x = pw->x1[1];
  const V x4 = pw->x1[4];
  const V xrow = pw->x16[256];

  // 16 bytes per thread and row; zero beyond the end (those outputs are not
  // stored, and only the last tile, whose aggregate nobody reads, has any)
  uint32_t w[kPfRows][4];
#pragma unroll
  for (int r = 0; r < kPfRows; ++r) {
    const uint64_t pos = base + r * kPfRow + (uint64_t)t * kPfBytes;
    w[r][0] = w[r][1] = w[r][2] = w[r][3] = 0;
    if (pos + kPfBytes <= n && ((reinterpret_cast<uintptr_t>(T) & 15) == 0)) {
      const uint4 v = *reinterpret_cast<const uint4*>(T + pos);
      w[r][0] = v.x; w[r][1] = v.y; w[r][2] = v.z; w[r][3] = v.w;
    } else {
      for (int k = 0; k < kPfBytes; ++k)
        if (pos + k < n) w[r][k >> 2] |= (uint32_t)T[pos + k] << (8 * (k & 3));
    }
  }
  const auto byte_at = [&](int r, int k) { return (V)((w[r][k >> 2] >> (8 * (k & 3))) & 0xFF); };

  // 1. thread aggregates: four 4-byte Horner chains per row joined with x^4;
  //    g[r][c] = the first c chains joined (g[r][0] = 0)
  V g[kPfRows][4];
  V E[kPfRows];
  V hrow[kPfRows];  // the thread's 16-byte fold per row
#pragma unroll
  for (int r = 0; r < kPfRows; ++r) {
    V hc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      V v = byte_at(r, 4 * c);
#pragma unroll
      for (int k = 1; k < 4; ++k) v = A::add(A::mul(v, x), byte_at(r, 4 * c + k));
      hc[c] = v;
    }
    g[r][0] = 0;
    g[r][1] = hc[0];
    g[r][2] = A::add(A::mul(g[r][1], x4), hc[1]);
    g[r][3] = A::add(A::mul(g[r][2], x4), hc[2]);
    const V h = A::add(A::mul(g[r][3], x4), hc[3]);
    hrow[r] = h;

    // 2. wave inclusive scan: I = sum_{u <= lane} h_u x^(16 (lane - u))
    V I = h;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const V o = __shfl_up(I, d);
      if (lane >= d) I = A::add(A::mul(o, pw->x16[d]), I);
    }
    V e = __shfl_up(I, 1);
    if (lane == 0) e = 0;
    E[r] = e;
    if (lane == 63) s_wave[r][wv] = I;
  }
  __syncthreads();
  // per row: prefix of the earlier waves (local) and the row aggregate; rows
  // fold into the tile aggregate, rp[r] = rows 0 .. r-1 of this tile
  V local[kPfRows], rp[kPfRows];
  V agg = 0;
#pragma unroll
  for (int r = 0; r < kPfRows; ++r) {
    V wp = 0, ra = 0;
#pragma unroll
    for (int v = 0; v < kPfThreads / 64; ++v) {
      if (v < wv) wp = A::add(A::mul(wp, pw->x16[64]), s_wave[r][v]);
      ra = A::add(A::mul(ra, pw->x16[64]), s_wave[r][v]);
    }
    local[r] = A::add(A::mul(wp, pw->x16[lane]), E[r]);
    rp[r] = agg;
    agg = A::add(A::mul(agg, xrow), ra);
  }

  // 3. carry-in from earlier tiles
  if (wv == 0) {
    V excl = 0;
    if (tile == 0) {
      if (lane == 0) st_relaxed(&status[0], A::kInc | (uint64_t)agg);
    } else {
      if (lane == 0) st_relaxed(&status[tile], A::kAgg | (uint64_t)agg);
      V mult = 1;
      int64_t look = (int64_t)tile - 1;
      while (true) {
        const int64_t pred = look - lane;
        uint64_t v = 0;
        if (pred >= 0) {
          do { v = ld_relaxed(&status[pred]); } while (!A::ready(v));
        }
        const uint64_t inc = __ballot(pred >= 0 && (v & A::kInc));
        const int stop = inc ? __ffsll((unsigned long long)inc) - 1 : 64;
        const V term = (lane <= stop && pred >= 0) ? A::mul(A::value(v), pw->xt[lane]) : (V)0;
        excl = A::add(excl, A::mul(A::wave_sum(term), mult));
        if (inc) break;
        mult = A::mul(mult, pw->xt[64]);
        look -= 64;
      }
      if (lane == 0)
        st_relaxed(&status[tile], A::kInc | (uint64_t)A::add(A::mul(excl, pw->xt[1]), agg));
    }
    if (lane == 0) s_excl = excl;
  }
  __syncthreads();

  // 4. outputs P[row + 16t + 1 .. row + 16t + 16], row by row
  V xr = 1;  // x^(row r)
  const V excl = s_excl;
  if (SAMPLED) {
#pragma unroll
    for (int r = 0; r < kPfRows; ++r) {
      const uint64_t pos = base + r * kPfRow + (uint64_t)t * kPfBytes;
      const V before_row = A::add(A::mul(excl, xr), rp[r]);
      const V C = A::add(A::mul(before_row, pw->x16[t]), local[r]);  // P[pos]
      if (pos <= n) P[pos >> 4] = C;
      if (pos + kPfBytes == n) P[n >> 4] = A::add(A::mul(C, pw->x16[1]), hrow[r]);
      xr = A::mul(xr, xrow);
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < kPfRows; ++r) {
    const uint64_t rowbase = base + r * kPfRow;
    const V before_row = A::add(A::mul(excl, xr), rp[r]);
    const V C = A::add(A::mul(before_row, pw->x16[t]), local[r]);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      V v = c ? A::add(A::mul(C, pw->x1[4 * c]), g[r][c]) : C;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        v = A::add(A::mul(v, x), byte_at(r, 4 * c + k));
        s_out[t * 17 + 4 * c + k] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPfBytes; ++q) {
      const uint64_t m = (uint64_t)t + (uint64_t)kPfThreads * q;
      if (rowbase + m < n) P[rowbase + 1 + m] = s_out[(m >> 4) * 17 + (m & 15)];
    }
    __syncthreads();  // s_out is reused by the next row
    xr = A::mul(xr, xrow);
  }
  if (tile == 0 && t == 0) P[0] = 0;
}

template <typename V>
__global__ void k_zero(V* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

template <class A, bool SAMPLED = false>
static hipError_t launch_prefix(const uint8_t* T, uint64_t n, typename A::V* P,
                                const typename A::Pow* pw, uint64_t* status, uint32_t* ctr,
                                hipStream_t s) {
  const uint64_t tiles = (n + kPfTile - 1) / kPfTile;
  if (tiles == 0) {
    // P[0] = 0 only
    k_zero<typename A::V><<<1, 64, 0, s>>>(P, 1);
    return hipGetLastError();
  }
  // status words and the tile counter
  const unsigned zb = (unsigned)((tiles + 255) / 256 < 4096 ? (tiles + 255) / 256 : 4096);
  k_zero<uint64_t><<<zb, 256, 0, s>>>(status, tiles);
  k_zero<uint32_t><<<1, 64, 0, s>>>(ctr, 1);
  k_prefix<A, SAMPLED><<<(unsigned)tiles, kPfThreads, 0, s>>>(T, n, P, pw, status, ctr);
  return hipGetLastError();
}

hipError_t launch_prefix_fp(const uint8_t* T, uint64_t n, uint64_t* P, const PfPow* pw,
                            uint64_t* status, uint32_t* ctr, hipStream_t s) {
  return launch_prefix<Mod61>(T, n, P, pw, status, ctr, s);
}

hipError_t launch_prefix_fp_sampled(const uint8_t* T, uint64_t n, uint64_t* Ps, const PfPow* pw,
                                    uint64_t* status, uint32_t* ctr, hipStream_t s) {
  return launch_prefix<Mod61, true>(T, n, Ps, pw, status, ctr, s);
}

hipError_t launch_prefix_h32(const uint8_t* T, uint64_t n, uint32_t* H, const PfPow32* pw,
                             uint64_t* status, uint32_t* ctr, hipStream_t s) {
  return launch_prefix<Mod32>(T, n, H, pw, status, ctr, s);
}

}  // namespace bt
