// The probe scan of a batch with text-local filters (Section 4.1, steps a4 and
// a6, for many texts at once).
//
// A batch's keys only ever match windows of their own text: each text's
// fingerprints carry their own salt, and a hit in another text counts as a
// collision.  One filter shared by every text of a phase would hold millions of
// keys and pass most windows; here each text has its own blocked filter of its
// keys' 32-bit hashes (one 32-bit word per key, three bits per key, set by
// k_keys), and a window is tested against its own text's filter only.
//
// Workgroups stay resident and take spans of span_chunks * kProbeTile
// consecutive window numbers from an atomic counter.  When a span's windows all
// belong to one text, the workgroup copies that text's filter into LDS (once
// per text: the next span of the same text keeps it) and tests there; a text
// whose filter is larger than LDS has a folded copy (each LDS word the OR of
// the words it covers), and a window that passes it is tested again against
// the full filter in global memory.  Spans that cross texts test each window
// against its text's filter in global memory (such texts are small, and so are
// their filters).  Inside a span, wave w takes chunks w, w + 16, ... of
// kProbeTile windows, laid out as in the shared-filter probe scan: in step k,
// lane l takes window chunk + 64 k + l, so consecutive lanes read consecutive
// prefix hashes.  The windows that pass join the per-wave candidate queue and
// probe the shared table 64 at a time with their 61-bit fingerprints.
#include "common.hpp"
#include "internal.hpp"
#include "lean.hpp"
#include "probe.hpp"
#include "window.hpp"

#include <type_traits>

namespace bt {

constexpr int kTlThreads = 1024;
constexpr uint32_t kTlWaves = kTlThreads / 64;
constexpr int kTlK = 16;  // windows per lane per chunk
// Windows per lane whose loads the dense fast path issues together, and the
// same for chunks that cross segments (each step's position kept).
constexpr int kTlGroup = 16;
constexpr int kTlSlowGroup = 4;
// Queue entries per wave: at most 63 wait between flushes and a step adds at
// most 63 more (indices up to 126), so 127 suffice; the byte this saves per
// wave leaves room for the workgroup's shared words beside a 64 KiB filter.
constexpr int kTlQueue = 127;
constexpr uint32_t kNoText = 0xFFFFFFFFu;
static_assert(64ull * kTlK == kProbeTile, "a chunk is one probe tile");
static_assert(kLeanK == kTlK, "lean chunks are probe tiles too");

// SEGT: where tiles cross many short segments (phase 2 of the lowest levels),
// a tile's segments are loaded once into registers and walked by shuffles; a
// separate instance, since the extra registers slow the other levels.
template <bool ODD, bool LEAN, bool SEGT>
__global__ __launch_bounds__(kTlThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_probe_text(PhaseArgs a, const uint64_t* __restrict__ woff, uint64_t span_chunks,
                  uint64_t* __restrict__ span_ctr, const uint64_t* __restrict__ span_info) {
  constexpr uint32_t FL = kTextFilterLdsLog2;
  extern __shared__ uint64_t s_lds[];
  uint32_t* s_filt = reinterpret_cast<uint32_t*>(s_lds);  // up to 2^FL words
  uint64_t* q = s_lds + (1u << (FL - 1)) + (uint64_t)(threadIdx.x >> 6) * kTlQueue;
  const uint64_t span = span_chunks * kProbeTile;
  __shared__ uint64_t s_span, s_r0, s_r1;
  __shared__ uint32_t s_text;    // the span's text when its filter goes to LDS, else kNoText
  __shared__ uint32_t s_loaded;  // the text whose filter LDS holds, or kNoText

  const int lane = lane_id();
  const uint32_t wave = threadIdx.x >> 6;
  uint32_t qn = 0;  // wave-uniform queue length

  const uint64_t R = a.lv.R;
  const uint64_t W = woff[R];
  const uint64_t* __restrict__ P = a.P;
  const uint32_t* __restrict__ H = a.P32;
  const uint64_t* __restrict__ rs_ = a.lv.rs;
  const uint64_t* __restrict__ re_ = a.lv.re;
  const uint64_t L = a.Lmain, xL = a.xLmain, fmask = a.fpmask;
  const uint32_t x32L = a.x32L;
  Slot* __restrict__ slots = a.tab.slots;
  const uint64_t mask = a.tab.mask;
  const uint32_t* __restrict__ tfw = a.tf_words;
  const uint64_t* __restrict__ tfo = a.tf_off;
  const uint32_t* __restrict__ tfl = a.tf_wl;
  // segments of the current span: [span_r0, span_r1]
  uint64_t span_r0 = 0, span_r1 = 0;

  const auto fp61 = [&](uint64_t i, uint64_t salt) {
    const uint64_t f = P ? sub61(P[i + L], mul61(P[i], xL)) : win61<true>(a, i, L, xL);
    return add61(f, salt) & fmask;
  };
  // the entry this lane holds: form its fingerprint and probe
  const auto probe_entry = [&](uint64_t e) {
    const uint64_t i = e & kQPosMask;
    probe(slots, mask, fp61(i, a.tx.tsalt[e >> kQPosBits]), i);
  };
  // whole wave: append the lanes' candidates; probe 64 once 64 are waiting
  uint64_t ncand = 0;  // wave-uniform: windows that passed the filters
  const auto push = [&](bool cand, uint64_t i, uint32_t t) {
    const uint64_t bal = __ballot(cand);
    if (!bal) return;
    const uint32_t my = (uint32_t)__popcll(bal & ((1ull << lane) - 1));
    if (cand) q[qn + my] = ((uint64_t)t << kQPosBits) | i;
    qn += (uint32_t)__popcll(bal);
    ncand += (uint64_t)__popcll(bal);
    if (qn >= 64) {
      wave_sync();
      const uint64_t e = q[lane];
      const bool mv = (uint32_t)lane < qn - 64;
      const uint64_t e2 = mv ? q[64 + lane] : 0;
      wave_sync();
      if (mv) q[lane] = e2;
      qn -= 64;
      probe_entry(e);
      wave_sync();
    }
  };

  // Memory-lean builds: lane l takes the kLeanK consecutive windows from
  // chunk + kLeanK l and rolls their hashes (lean.hpp).
  const auto scan_chunk_lean = [&](uint64_t ch, auto lds_tag, uint32_t st, uint32_t lwl, bool big) {
    constexpr bool LDS = decltype(lds_tag)::value;
    uint64_t toff = LDS ? tfo[st] : 0;
    uint32_t twl = LDS ? tfl[st] : 0;
    const auto on_text = [&](uint32_t t) {
      if (!LDS) {
        toff = tfo[t];
        twl = tfl[t];
      }
    };
    const auto pass_word = [&](uint32_t h) -> uint32_t {
      return LDS ? s_filt[tfilter_word(h, lwl)] : tfw[toff + tfilter_word(h, twl)];
    };
    const auto test8 = [&](const uint32_t* hv, bool* ok) {
      uint32_t wv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) wv[k] = pass_word(hv[k]);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t m = tfilter_mask(hv[k]);
        ok[k] = (wv[k] & m) == m;
      }
      if (LDS && big) {
#pragma unroll
        for (int k = 0; k < 8; ++k) wv[k] = ok[k] ? tfw[toff + tfilter_word(hv[k], twl)] : 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t m = tfilter_mask(hv[k]);
          ok[k] = ok[k] && (wv[k] & m) == m;
        }
      }
    };
    const auto test1 = [&](uint32_t h) {
      const uint32_t m = tfilter_mask(h);
      bool c = (pass_word(h) & m) == m;
      if (LDS && big && c) c = (tfw[toff + tfilter_word(h, twl)] & m) == m;
      return c;
    };
    lean_chunk<ODD, true, true>(a, woff, span_r0, span_r1 + 1, W,
                                ch * kProbeTile + (uint64_t)lane * kLeanK, on_text, test8, test1,
                                push);
  };

  // One chunk of kProbeTile window numbers.  LDS (a compile-time tag): every
  // window of the chunk belongs to text st, whose filter (2^lwl words, lwl =
  // its word count or the folded one) is in LDS; when folded (big), a window
  // that passes is tested again against the full filter.  Otherwise each lane
  // reads its own text's filter in global memory.
  const auto scan_chunk = [&](uint64_t ch, auto lds_tag, uint32_t st, uint32_t lwl, bool big) {
    constexpr bool LDS = decltype(lds_tag)::value;
    if constexpr (LEAN) {
      scan_chunk_lean(ch, lds_tag, st, lwl, big);
      return;
    }
    const uint64_t w0 = ch * kProbeTile + lane;
    uint64_t r = segment_in(woff, span_r0, span_r1 + 1, w0);
    uint64_t wo = woff[r], wn = woff[r + 1], rs = rs_[r], re = re_[r];
    // lanes past the last window hold no segment: they read no text entry
    uint32_t t = w0 < W ? a.lv.rtext[r] : 0;
    uint64_t salt = a.tx.tsalt[t];
    uint64_t toff = tfo[LDS ? st : t];
    uint32_t twl = tfl[LDS ? st : t];
    const auto pass_word = [&](uint32_t h) -> uint32_t {
      return LDS ? s_filt[tfilter_word(h, lwl)] : tfw[toff + tfilter_word(h, twl)];
    };
    // the text's short final key, if any (kept in registers while t holds)
    uint64_t oL = 0, opos = 0;
    uint32_t oh = 0, ox = 0;
    const auto load_odd = [&]() {
      oL = a.odd.L[t];
      if (oL) {
        opos = a.odd.pos[t];
        const uint64_t hx = a.odd.h32[t];
        oh = (uint32_t)hx;
        ox = (uint32_t)(hx >> 32);
      }
    };
    if (ODD && w0 < W) load_odd();
    // the short key's 61-bit fingerprint at i, against the key's (text t)
    const auto odd61 = [&](uint64_t i, uint64_t sl) {
      uint64_t g = P ? sub61(P[i + oL], mul61(P[i], a.odd.xp[t])) : win61<true>(a, i, oL, a.odd.xp[t]);
      g = add61(g, sl);
      if ((g & fmask) == a.odd.fp[t] && i < a.odd.best[t])
        atomicMin((unsigned long long*)&a.odd.best[t], (unsigned long long)i);
    };

    // every lane's 16 windows inside its segment: eight steps' loads at once
    {
      const uint64_t wl = w0 + 64ull * (kTlK - 1);
      const bool lane_ok = wl < wn && rs + (wl - wo) + L <= re;
      if (__ballot(lane_ok) == ~0ull) {
        const uint64_t i0 = rs + (w0 - wo);
        const uint32_t s32 = (uint32_t)salt;
#pragma unroll
        for (int k0 = 0; k0 < kTlK; k0 += kTlGroup) {
          // the group's loads (two per window, three with a short key) leave
          // together: the scheduler would otherwise pair each load with its
          // use and wait out every latency in turn
          uint32_t ha[kTlGroup], hb[kTlGroup], hc[kTlGroup];
          // (and the short key's, H[i + oL], where the text has one)
          const bool oddk = ODD && oL;
#pragma unroll
          for (int k = 0; k < kTlGroup; ++k) {
            const uint64_t i = i0 + 64ull * (k0 + k);
            hb[k] = H[i + L];
            ha[k] = H[i];
            if (oddk) hc[k] = H[i + oL];
          }
          __builtin_amdgcn_sched_barrier(0);
          uint32_t hv[kTlGroup];
#pragma unroll
          for (int k = 0; k < kTlGroup; ++k) hv[k] = hb[k] - ha[k] * x32L + s32;
          if (oddk) {
            // the short key's 32-bit hashes (loaded with the others); the rare
            // matches form their 61-bit fingerprints one at a time
            uint32_t om = 0;
#pragma unroll
            for (int k = 0; k < kTlGroup; ++k) {
              const uint64_t i = i0 + 64ull * (k0 + k);
              if (i < opos && hc[k] - ha[k] * ox + s32 == oh) om |= 1u << k;
            }
            while (om) {
              const int k = __builtin_ctz(om);
              om &= om - 1;
              odd61(i0 + 64ull * (k0 + k), salt);
            }
          }
          uint32_t wv[kTlGroup];
#pragma unroll
          for (int k = 0; k < kTlGroup; ++k) wv[k] = pass_word(hv[k]);
          bool ok[kTlGroup];
#pragma unroll
          for (int k = 0; k < kTlGroup; ++k) {
            const uint32_t m = tfilter_mask(hv[k]);
            ok[k] = (wv[k] & m) == m;
          }
          if (LDS && big) {
            // passed the folded filter: the full one, the loads issued together
#pragma unroll
            for (int k = 0; k < kTlGroup; ++k) wv[k] = ok[k] ? tfw[toff + tfilter_word(hv[k], twl)] : 0u;
#pragma unroll
            for (int k = 0; k < kTlGroup; ++k) {
              const uint32_t m = tfilter_mask(hv[k]);
              ok[k] = ok[k] && (wv[k] & m) == m;
            }
          }
#pragma unroll
          for (int k = 0; k < kTlGroup; ++k) push(ok[k], i0 + 64ull * (k0 + k), t);
        }
        return;
      }
    }

    if constexpr (LDS) {
      // The chunk crosses segments, all of the span's one text (salt, filter
      // and short key stay).  Per group of steps each lane first follows its
      // windows across the segments, then the group's loads leave together.
      const uint32_t s32 = (uint32_t)salt;
      // (SEGT) the segments from lane 0's on, segment rb + s in lane s: its
      // end as a window number relative to the tile (clamped) and its
      // positions; past the 64th, a lane reads global memory
      const uint64_t cw = ch * kProbeTile;
      uint64_t rb = 0, trs = 0, tre = 0;
      uint32_t tend = ~0u;
      if constexpr (SEGT) {
        rb = shfl64(r, 0);
        const uint64_t q = rb + (uint64_t)lane;
        if (q < R) {
          const uint64_t e = woff[q + 1] - cw;
          tend = e < 0xFFFFFFFFull ? (uint32_t)e : ~0u;
          trs = rs_[q];
          tre = re_[q];
        }
      }
#pragma unroll
      for (int k0 = 0; k0 < kTlK; k0 += kTlSlowGroup) {
        uint64_t ik[kTlSlowGroup];
        uint32_t vm = 0, om = 0;  // steps with a main-length window, with a short-key window
#pragma unroll
        for (int k = 0; k < kTlSlowGroup; ++k) {
          const uint64_t w = w0 + 64ull * (k0 + k);
          const bool live = w < W;
          if constexpr (SEGT) {
            bool adv = live && w >= wn;
            while (__ballot(adv)) {
              // every lane takes part in the shuffles; those moving on use them
              const uint64_t s = r + 1 - rb;
              const uint32_t sl = (uint32_t)s & 63u;
              const uint32_t ne = __shfl(tend, (int)sl);
              const uint64_t nrs = shfl64(trs, sl), nre = shfl64(tre, sl);
              if (adv) {
                ++r;
                wo = wn;
                if (s < 64) {
                  wn = cw + ne;
                  rs = nrs;
                  re = nre;
                } else {
                  wn = woff[r + 1];
                  rs = rs_[r];
                  re = re_[r];
                }
                adv = w >= wn;
              }
            }
          } else if (live && w >= wn) {
            do {
              ++r;
              wo = wn;
              wn = woff[r + 1];
            } while (w >= wn);
            rs = rs_[r];
            re = re_[r];
          }
          const uint64_t i = rs + (w - wo);
          ik[k] = i;
          if (live && i + L <= re) vm |= 1u << k;
          if (ODD && live && oL && i + oL <= re && i < opos) om |= 1u << k;
        }
        uint32_t ha[kTlSlowGroup], hb[kTlSlowGroup], hc[kTlSlowGroup];
#pragma unroll
        for (int k = 0; k < kTlSlowGroup; ++k) {
          hb[k] = ((vm >> k) & 1) ? H[ik[k] + L] : 0u;
          ha[k] = (((vm | om) >> k) & 1) ? H[ik[k]] : 0u;
          if (ODD) hc[k] = ((om >> k) & 1) ? H[ik[k] + oL] : 0u;
        }
        __builtin_amdgcn_sched_barrier(0);
        if (ODD) {
          uint32_t mm = 0;
#pragma unroll
          for (int k = 0; k < kTlSlowGroup; ++k)
            if (((om >> k) & 1) && hc[k] - ha[k] * ox + s32 == oh) mm |= 1u << k;
          while (mm) {
            const int k = __builtin_ctz(mm);
            mm &= mm - 1;
            odd61(ik[k], salt);
          }
        }
        uint32_t hv[kTlSlowGroup], wv[kTlSlowGroup];
        bool ok[kTlSlowGroup];
#pragma unroll
        for (int k = 0; k < kTlSlowGroup; ++k) {
          hv[k] = hb[k] - ha[k] * x32L + s32;
          wv[k] = ((vm >> k) & 1) ? pass_word(hv[k]) : 0u;
        }
#pragma unroll
        for (int k = 0; k < kTlSlowGroup; ++k) {
          const uint32_t m = tfilter_mask(hv[k]);
          ok[k] = ((vm >> k) & 1) && (wv[k] & m) == m;
        }
        if (big) {
#pragma unroll
          for (int k = 0; k < kTlSlowGroup; ++k) wv[k] = ok[k] ? tfw[toff + tfilter_word(hv[k], twl)] : 0u;
#pragma unroll
          for (int k = 0; k < kTlSlowGroup; ++k) {
            const uint32_t m = tfilter_mask(hv[k]);
            ok[k] = ok[k] && (wv[k] & m) == m;
          }
        }
#pragma unroll
        for (int k = 0; k < kTlSlowGroup; ++k) push(ok[k], ik[k], t);
      }
      return;
    }

    // per step, following each lane across segment (and text) boundaries
    for (int k = 0; k < kTlK; ++k) {
      const uint64_t w = w0 + (uint64_t)k * 64;
      const bool live = w < W;  // every lane stays in the loop (the queue is wave-wide)
      if (live && w >= wn) {
        do {
          ++r;
          wo = wn;
          wn = woff[r + 1];
        } while (w >= wn);
        rs = rs_[r];
        re = re_[r];
        t = a.lv.rtext[r];
        salt = a.tx.tsalt[t];
        if (!LDS) {
          toff = tfo[t];
          twl = tfl[t];
        }
        if (ODD) load_odd();
      }
      const uint64_t i = rs + (w - wo);
      bool cand = false;
      if (live && i + L <= re) {
        const uint32_t h = H[i + L] - H[i] * x32L + (uint32_t)salt;
        const uint32_t m = tfilter_mask(h);
        cand = (pass_word(h) & m) == m;
        if (LDS && big && cand) cand = (tfw[toff + tfilter_word(h, twl)] & m) == m;
      }
      push(cand, i, t);
      // the short key: its 32-bit hash first (equal strings always agree),
      // the 61-bit fingerprint only where that matches
      if (ODD && live && oL && i + oL <= re && i < opos) {
        const uint32_t ho = H[i + oL] - H[i] * ox + (uint32_t)salt;
        if (ho == oh) odd61(i, salt);
      }
    }
  };

  if (threadIdx.x == 0) s_loaded = kNoText;
  while (true) {
    __syncthreads();  // the previous span is done with s_filt and s_span
    if (threadIdx.x == 0) {
      const uint64_t sp = atomicAdd((unsigned long long*)span_ctr, 1ull);
      if (sp * span < W) {
        s_r0 = span_info[3 * sp];
        s_r1 = span_info[3 * sp + 1];
        s_text = (uint32_t)span_info[3 * sp + 2];
      }
      s_span = sp;
    }
    __syncthreads();
    const uint64_t sp = s_span;
    if (sp * span >= W) break;
    const uint32_t st = s_text;
    span_r0 = s_r0;
    span_r1 = s_r1;
    if (st != kNoText) {
      const uint32_t wl = tfl[st];
      const bool big = wl > FL;
      const uint32_t lwl = big ? FL : wl;
      if (st != s_loaded) {
        // 2^lwl >= 8 words: whole 16-byte groups
        const uint64_t ng = (1ull << lwl) / 4;
        const uint4* src = reinterpret_cast<const uint4*>(big ? a.tf_fold + a.tf_fold_off[st]
                                                              : tfw + tfo[st]);
        uint4* dst = reinterpret_cast<uint4*>(s_filt);
        for (uint64_t k = threadIdx.x; k < ng; k += kTlThreads) dst[k] = src[k];
        __syncthreads();
        if (threadIdx.x == 0) s_loaded = st;
      }
      for (uint64_t c = wave; c < span_chunks; c += kTlWaves) {
        const uint64_t ch = sp * span_chunks + c;
        if (ch * kProbeTile >= W) break;
        scan_chunk(ch, std::true_type{}, st, lwl, big);
      }
    } else {
      for (uint64_t c = wave; c < span_chunks; c += kTlWaves) {
        const uint64_t ch = sp * span_chunks + c;
        if (ch * kProbeTile >= W) break;
        scan_chunk(ch, std::false_type{}, 0u, 0u, false);
      }
    }
  }
  if (qn) {
    wave_sync();
    if ((uint32_t)lane < qn) probe_entry(q[lane]);
  }
  if (a.pc && lane == 0 && ncand) atomicAdd((unsigned long long*)(a.pc + kPcCand), (unsigned long long)ncand);
}

// Per span of `span` window numbers (those below W): its first and last
// segment and, when both belong to one text, that text (else kNoText), as
// three words.  One thread per span, so that the resident workgroups of the
// scan read a span's facts with one load instead of searching for them.
__global__ void k_span_info(const uint64_t* __restrict__ woff, uint64_t R,
                            const uint32_t* __restrict__ rtext, uint64_t span, uint64_t nspan,
                            uint64_t* __restrict__ info) {
  const uint64_t W = woff[R];
  for (uint64_t sp = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; sp < nspan;
       sp += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t w0 = sp * span;
    if (w0 >= W) break;
    const uint64_t w1 = (W - w0 < span ? W : w0 + span) - 1;
    const uint64_t r0 = segment_of(woff, R, w0), r1 = segment_in(woff, r0, R, w1);
    const uint32_t t0 = rtext[r0], t1 = rtext[r1];
    info[3 * sp] = r0;
    info[3 * sp + 1] = r1;
    info[3 * sp + 2] = t0 == t1 ? t0 : kNoText;
  }
}

uint64_t probe_text_spans(uint64_t max_windows, uint64_t span_chunks) {
  const uint64_t span = span_chunks * kProbeTile;
  return (max_windows + span - 1) / span;
}

hipError_t launch_span_info(const PhaseArgs& a, const uint64_t* woff, uint64_t max_windows,
                            uint64_t span_chunks, uint64_t* span_info, hipStream_t s) {
  if (a.lv.R == 0) return hipSuccess;
  if (span_chunks == 0 || !span_info) return hipErrorInvalidValue;
  const uint64_t spans = probe_text_spans(max_windows, span_chunks);
  const uint64_t g = (spans + 255) / 256;
  k_span_info<<<(unsigned)(g < 4096 ? (g ? g : 1) : 4096), 256, 0, s>>>(
      woff, a.lv.R, a.lv.rtext, span_chunks * kProbeTile, spans, span_info);
  return hipGetLastError();
}

hipError_t launch_probe_text(const PhaseArgs& a, const uint64_t* woff, bool has_odd,
                             uint64_t max_windows, uint64_t span_chunks, uint64_t* span_ctr,
                             const uint64_t* span_info, bool short_segments, hipStream_t s) {
  if (a.lv.R == 0) return hipSuccess;
  if (!a.tf_words || !a.pre32 || span_chunks == 0 || !span_info) return hipErrorInvalidValue;
  const uint64_t spans = probe_text_spans(max_windows, span_chunks);
  // one resident 1024-thread workgroup per CU (256 CUs): registers (up to 128
  // VGPRs) and LDS (128 KiB of filter plus the queues) allow one
  const unsigned grid = (unsigned)(spans < 256 ? (spans ? spans : 1) : 256);
  const bool lean = a.P32 == nullptr;  // sampled 32-bit hashes: the rolled window loop
  const size_t lds = ((size_t)4 << kTextFilterLdsLog2) + (size_t)kTlWaves * kTlQueue * 8;
#define BT_TL_LAUNCH(O, LN, SG)                                                             \
  do {                                                                                      \
    const hipError_t e = hipFuncSetAttribute(                                               \
        reinterpret_cast<const void*>(&k_probe_text<O, LN, SG>),                            \
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                              \
    if (e != hipSuccess) return e;                                                          \
    k_probe_text<O, LN, SG><<<grid, kTlThreads, lds, s>>>(a, woff, span_chunks, span_ctr,     \
                                                         span_info);                        \
  } while (0)
  const bool segt = short_segments && !lean;
  if (has_odd) {
    if (lean) BT_TL_LAUNCH(true, true, false);
    else if (segt) BT_TL_LAUNCH(true, false, true);
    else BT_TL_LAUNCH(true, false, false);
  } else {
    if (lean) BT_TL_LAUNCH(false, true, false);
    else if (segt) BT_TL_LAUNCH(false, false, true);
    else BT_TL_LAUNCH(false, false, false);
  }
#undef BT_TL_LAUNCH
  return hipGetLastError();
}

// Word k of text big[b]'s folded filter: the OR of the 2^d full-filter words
// k 2^d .. (k + 1) 2^d - 1, d = wl - F (F = kTextFilterLdsLog2).
// A window's folded word index is its full index shifted right by d (both
// take the top bits of the same product), so the fold passes every window the
// full filter passes.
__global__ void k_fold_filters(PhaseArgs a, const uint32_t* __restrict__ big, uint32_t nbig,
                               uint32_t F) {
  const uint64_t per = 1ull << F;
  const uint64_t n = (uint64_t)nbig * per;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t t = big[i >> F];
    const uint64_t k = i & (per - 1);
    const uint32_t d = a.tf_wl[t] - F;
    const uint32_t* src = a.tf_words + a.tf_off[t] + (k << d);
    uint32_t v = 0;
    for (uint64_t j = 0; j < (1ull << d); ++j) v |= src[j];
    a.tf_fold[a.tf_fold_off[t] + k] = v;
  }
}

hipError_t launch_fold_filters(const PhaseArgs& a, const uint32_t* big, uint32_t nbig,
                               hipStream_t s) {
  if (!nbig) return hipSuccess;
  const uint32_t F = kTextFilterLdsLog2;
  const uint64_t n = (uint64_t)nbig << F;
  const uint64_t g = (n + 255) / 256;
  k_fold_filters<<<(unsigned)(g < 8192 ? g : 8192), 256, 0, s>>>(a, big, nbig, F);
  return hipGetLastError();
}

}  // namespace bt
