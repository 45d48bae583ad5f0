// The memory-lean probe scan's window loop (lean_chunk) run on the CPU: 64
// threads play one wave's lanes over random texts, runs and segments (empty
// segments, gaps, windows whose main length does not fit, texts starting at
// position 0).  Checks: every window whose main window fits is tested exactly
// once, with the 32-bit hash H[i+L] - H[i] x^L (+ salt) computed directly; the
// short final key's leftmost scanned occurrence equals brute force; and every
// access stays inside exact-size heap arrays (built with AddressSanitizer).
//   lean_scan_host SEED   (exit status 0 when every trial passes)
#include "lean.hpp"
#include <cstdio>
#include <cstring>
#include <random>
#include <thread>
#include <vector>
#include <mutex>
thread_local dim3_ threadIdx;
std::barrier<>* g_bar;
bool g_pred[64];
using namespace bt;

static uint64_t hmad61(uint64_t a, uint64_t b, uint64_t c) {
  return (uint64_t)(((unsigned __int128)a * b + c) % kP61);
}

int main(int argc, char** argv) {
  int seed = argc > 1 ? atoi(argv[1]) : 1;
  std::mt19937_64 rng(seed);
  int fails = 0;
  for (int trial = 0; trial < 40; ++trial) {
    const uint64_t base = rng() % 37;
    const uint64_t n = 200 + rng() % 6000;
    const uint64_t end = base + n;
    const int sig = 1 + rng() % 4;
    const uint64_t per = 1 + rng() % 90;
    uint8_t* T = new uint8_t[end];
    for (uint64_t i = 0; i < end; ++i) T[i] = (uint8_t)(rng() % 256);
    for (uint64_t i = base; i < end; ++i)
      T[i] = (trial & 1) ? (uint8_t)('a' + ((i - base) % per) % sig) : (uint8_t)('a' + rng() % sig);
    const uint32_t x32 = (uint32_t)rng() | 1u;
    const uint64_t x = 1000 + rng() % (kP61 - 2000);
    // prefix arrays (dense, then sampled copies of exact size)
    std::vector<uint32_t> H(n + 1);
    std::vector<uint64_t> P(n + 1);
    H[0] = 0; P[0] = 0;
    for (uint64_t i = 0; i < n; ++i) {
      H[i + 1] = H[i] * x32 + T[base + i];
      P[i + 1] = hmad61(P[i], x, T[base + i]);
    }
    const uint64_t ns = n / 16 + 1;
    uint32_t* Hs = new uint32_t[ns];
    uint64_t* Ps = new uint64_t[ns];
    for (uint64_t q = 0; q < ns; ++q) { Hs[q] = H[16 * q]; Ps[q] = P[16 * q]; }
    const uint64_t L = 1 + rng() % 80;
    const uint64_t oL = (rng() % 3 == 0 || L == 1) ? 0 : 1 + rng() % (L - 1);
    const uint64_t Lmin = oL ? oL : L;
    // segments: runs [rs, re) with a window range each, windows counted as the
    // builds count them (starts whose shortest window fits)
    std::vector<uint64_t> vrs, vre, vcnt;
    std::vector<uint32_t> vtx;
    uint64_t p = base;
    while (p < end) {
      const uint64_t runend = std::min<uint64_t>(end, p + 1 + rng() % 700);
      uint64_t s = p;
      while (s < runend) {
        const uint64_t e2 = std::min<uint64_t>(runend, s + 1 + rng() % 300);
        // a segment: starts s .. e2-1 (limited by the run end), maybe empty
        uint64_t cnt = 0;
        if (runend >= Lmin + s) cnt = std::min<uint64_t>(e2 - s, runend - Lmin - s + 1);
        if (rng() % 5 == 0) cnt = 0;
        vrs.push_back(s); vre.push_back(runend); vcnt.push_back(cnt); vtx.push_back(0);
        s = e2 + (rng() % 4 == 0 ? rng() % 50 : 0);
      }
      p = runend + (rng() % 3 == 0 ? rng() % 40 : 0);
    }
    const uint64_t R = vrs.size();
    uint64_t* woff = new uint64_t[R + 1];
    woff[0] = 0;
    for (uint64_t r = 0; r < R; ++r) woff[r + 1] = woff[r] + vcnt[r];
    const uint64_t W = woff[R];
    uint64_t* rs = new uint64_t[R];
    uint64_t* re = new uint64_t[R];
    uint32_t* rtext = new uint32_t[R];
    for (uint64_t r = 0; r < R; ++r) { rs[r] = vrs[r]; re[r] = vre[r]; rtext[r] = 0; }
    uint64_t* tsalt = new uint64_t[1];
    tsalt[0] = (trial & 2) ? (rng() % kP61) : 0;
    // the short key: a window of length oL near the end
    uint64_t* oLp = new uint64_t[1];
    uint64_t* oxp = new uint64_t[1];
    uint64_t* ofp = new uint64_t[1];
    uint64_t* obest = new uint64_t[1];
    uint64_t* opos = new uint64_t[1];
    uint64_t* onk = new uint64_t[1];
    uint64_t* oh32 = new uint64_t[1];
    oLp[0] = oL;
    uint64_t kpos = 0;
    if (oL) {
      kpos = end - oL;
      uint64_t xp = 1;
      uint32_t x32p = 1;
      for (uint64_t k = 0; k < oL; ++k) { xp = hmad61(xp, x, 0); x32p *= x32; }
      const uint64_t f = (P[kpos - base + oL] + kP61 - hmad61(P[kpos - base], xp, 0)) % kP61;
      oxp[0] = xp;
      ofp[0] = (f + tsalt[0]) % kP61;
      obest[0] = kpos;
      opos[0] = kpos;
      const uint32_t h = H[kpos - base + oL] - H[kpos - base] * x32p + (uint32_t)tsalt[0];
      oh32[0] = (uint64_t)h | ((uint64_t)x32p << 32);
    }
    onk[0] = 1;
    PhaseArgs a{};
    a.T = T; a.Ps = Ps; a.pshift = 4; a.Hs = Hs; a.pbase = base; a.pend = end; a.x = x;
    a.Lmain = L; a.fpmask = ~0ull; a.x32 = x32;
    uint32_t xl = 1; for (uint64_t k = 0; k < L; ++k) xl *= x32;
    uint32_t xlm1 = 1; for (uint64_t k = 0; k + 1 < L; ++k) xlm1 *= x32;
    uint32_t inv = x32; for (int k = 0; k < 4; ++k) inv *= 2u - x32 * inv;
    a.x32L = xl; a.x32Lm1 = xlm1; a.x32inv = inv;
    a.lv.R = R; a.lv.rs = rs; a.lv.re = re; a.lv.rtext = rtext;
    a.tx.T = 1; a.tx.tsalt = tsalt;
    a.odd = OddDev{oLp, oxp, ofp, obest, opos, onk, oh32};
    // run: 64 lane threads, chunks of 1024 window numbers
    std::vector<uint8_t> seen(W, 0);
    std::mutex mu;
    int bad = 0;
    std::barrier<> bar(64);
    g_bar = &bar;
    auto lane_fn = [&](int lane) {
      threadIdx.x = lane;
      for (uint64_t ch = 0; ch * 1024 < W; ++ch) {
        std::vector<uint32_t> fifo;
        const auto on_text = [](uint32_t) {};
        const auto test8 = [&](const uint32_t* hv, bool* ok) {
          for (int k = 0; k < 8; ++k) { fifo.push_back(hv[k]); ok[k] = true; }
        };
        const auto test1 = [&](uint32_t h) { fifo.push_back(h); return true; };
        size_t fi = 0;
        const auto push = [&](bool cand, uint64_t i, uint32_t t) {
          if (!cand) return;
          const uint32_t h = fifo.at(fi++);
          const uint32_t want = H[i - base + L] - H[i - base] * xl + (uint32_t)tsalt[0];
          std::lock_guard<std::mutex> g(mu);
          if (h != want) { if (bad < 5) printf("trial %d: window %lu hash %08x want %08x\n", trial, i, h, want); ++bad; }
          // find the window number
          uint64_t r = 0;
          while (!(i >= rs[r] && i < rs[r] + (woff[r + 1] - woff[r]) && woff[r + 1] > woff[r])) ++r;
          seen[woff[r] + (i - rs[r])]++;
        };
        lean_chunk<true, true, true>(a, woff, 0, R, W, ch * 1024 + (uint64_t)lane * kLeanK, on_text,
                                     test8, test1, push);
        if (fi != fifo.size()) { std::lock_guard<std::mutex> g(mu); ++bad; printf("fifo mismatch\n"); }
      }
    };
    std::vector<std::thread> th;
    for (int l = 0; l < 64; ++l) th.emplace_back(lane_fn, l);
    for (auto& t : th) t.join();
    // every window whose main window fits was tested exactly once
    for (uint64_t r = 0; r < R; ++r)
      for (uint64_t w = woff[r]; w < woff[r + 1]; ++w) {
        const uint64_t i = rs[r] + (w - woff[r]);
        const int want = i + L <= re[r] ? 1 : 0;
        if (seen[w] != want) { if (bad < 5) printf("trial %d: window %lu seen %d want %d\n", trial, i, seen[w], want); ++bad; }
      }
    // the short key's leftmost occurrence among the scanned starts before it
    if (oL) {
      uint64_t best = kpos;
      for (uint64_t r = 0; r < R; ++r)
        for (uint64_t w = woff[r]; w < woff[r + 1]; ++w) {
          const uint64_t i = rs[r] + (w - woff[r]);
          if (i < kpos && i + oL <= re[r] && i < best && memcmp(T + i, T + kpos, oL) == 0) best = i;
        }
      if (obest[0] != best) { printf("trial %d: short key best %lu want %lu\n", trial, obest[0], best); ++bad; }
    }
    if (bad) { printf("trial %d (n %lu L %lu oL %lu R %lu W %lu): %d bad\n", trial, n, L, oL, R, W, bad); ++fails; }
    delete[] T; delete[] Hs; delete[] Ps; delete[] woff; delete[] rs; delete[] re; delete[] rtext;
    delete[] tsalt; delete[] oLp; delete[] oxp; delete[] ofp; delete[] obest; delete[] opos; delete[] onk; delete[] oh32;
  }
  printf("seed %d: %d failing trials\n", seed, fails);
  return fails != 0;
}
