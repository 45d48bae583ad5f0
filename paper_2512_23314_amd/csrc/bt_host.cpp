// libbt host side: the C ABI of include/bt.h, the device memory pool, and the
// level loop that drives the kernels of level.hip.
//
// Build, for one or many texts (a single text is a batch of one):
//   - plan every text: b1 = leaf * tau^k (k from s_hint or root_block_len),
//     h = k + 1 levels;
//   - prefix fingerprints of the whole concatenation, once (step a2);
//   - steps s = 0 .. H-1 with block length b = leaf * tau^(H-1-s): a text whose
//     b1 equals b enters with its level-1 blocks, every other present text
//     continues with the children of its marked blocks; all present texts go
//     through the same launches (phase 1, marks, phase 2, pointers, split);
//   - the last step (b = leaf) stores the leaf bytes.
// Texts in one build never match each other: each text's fingerprints get a
// per-text salt, and a candidate occurrence outside the key's own text counts
// as a collision.
//
// Collision fallback (why a retry can start just past the false hit): let best
// be the smallest window position whose fingerprint equals the key's, and let
// its bytes differ from the key.  The true leftmost occurrence p* lies inside a
// run (see level.hip), so its window was probed and fingerprints equal:
// best <= p*, and best != p*.  Hence no true occurrence lies in [best, p*) or
// before best, and a walk over all text positions from best + 1 that verifies
// each fingerprint hit finds p* first.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "bt.h"
#include "internal.hpp"
#include "query.hpp"

namespace bt {

// ------------------------------------------------------------------ pool

// Device memory of a context: blocks from the caller's allocator (bt_allocator)
// or hipMalloc, kept on a free list when returned and reused by size; trim()
// gives the cached ones back.
class Pool {
 public:
  Pool(int dev, const bt_allocator* a, hipStream_t s) : dev_(dev), stream_(s) {
    if (a) {
      ext_ = *a;
      has_ext_ = true;
    }
  }
  ~Pool() {
    trim();
    for (auto& kv : size_) release(kv.first);  // leaked buffers (trees outliving everything)
  }
  void* get(size_t bytes) {
    if (bytes == 0) bytes = 1;
    const size_t want = round(bytes);
    std::lock_guard<std::mutex> g(mu_);
    auto it = free_.lower_bound(want);
    if (it != free_.end() && it->first <= want + want / 4) {
      void* p = it->second;
      in_use_ += it->first;
      if (in_use_ > peak_) peak_ = in_use_;
      free_.erase(it);
      return p;
    }
    int old = -1;
    (void)hipGetDevice(&old);
    if (old != dev_) (void)hipSetDevice(dev_);
    void* p = acquire(want);
    if (!p) {
      // release cached blocks and try once more
      for (auto& kv : free_) {
        release(kv.second);
        held_ -= size_[kv.second];
        size_.erase(kv.second);
      }
      free_.clear();
      p = acquire(want);
    }
    if (old != dev_ && old >= 0) (void)hipSetDevice(old);
    if (!p) return nullptr;
    size_[p] = want;
    held_ += want;
    in_use_ += want;
    if (in_use_ > peak_) peak_ = in_use_;
    return p;
  }
  void put(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu_);
    auto it = size_.find(p);
    if (it == size_.end()) return;
    in_use_ -= it->second;
    free_.emplace(it->second, p);
  }
  void trim() {
    std::lock_guard<std::mutex> g(mu_);
    for (auto& kv : free_) {
      release(kv.second);
      held_ -= size_[kv.second];
      size_.erase(kv.second);
    }
    free_.clear();
  }
  uint64_t held() const { return held_; }
  // bytes handed out and not returned; the most of that since reset_peak()
  uint64_t in_use() const { return in_use_; }
  uint64_t peak() const { return peak_; }
  void reset_peak() {
    std::lock_guard<std::mutex> g(mu_);
    peak_ = in_use_;
  }

 private:
  static size_t round(size_t b) {
    if (b <= (1u << 20)) {
      size_t r = 256;
      while (r < b) r <<= 1;
      return r;
    }
    const size_t g = 2u << 20;
    return (b + g - 1) / g * g;
  }
  // one block from the caller's allocator or hipMalloc; null on failure
  void* acquire(size_t bytes) {
    if (has_ext_) return ext_.alloc(ext_.user, bytes, stream_);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void release(void* p) {
    if (has_ext_) ext_.free(ext_.user, p, stream_);
    else (void)hipFree(p);
  }
  int dev_;
  hipStream_t stream_;
  bt_allocator ext_{};
  bool has_ext_ = false;
  std::mutex mu_;
  std::multimap<size_t, void*> free_;
  std::unordered_map<void*, size_t> size_;
  uint64_t held_ = 0, in_use_ = 0, peak_ = 0;
};

template <typename T>
struct Buf {
  std::shared_ptr<Pool> pool;
  T* p = nullptr;
  uint64_t n = 0;
  Buf() = default;
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  Buf(Buf&& o) noexcept : pool(std::move(o.pool)), p(o.p), n(o.n) { o.p = nullptr; }
  Buf& operator=(Buf&& o) noexcept {
    reset();
    pool = std::move(o.pool);
    p = o.p;
    n = o.n;
    o.p = nullptr;
    return *this;
  }
  ~Buf() { reset(); }
  void reset() {
    if (p && pool) pool->put(p);
    p = nullptr;
    n = 0;
  }
  T* release() {
    T* q = p;
    p = nullptr;
    return q;
  }
};

}  // namespace bt

using namespace bt;

// ------------------------------------------------------------------ fixed scratch
//
// bt_prefix_scan_noalloc keeps the prefix scan's scratch -- the power tables and
// the look-back status words -- in this fixed device array instead of the
// context's pool, so that the call allocates nothing.  Each GPU holds its own
// copy until the process ends.  In host code the array's name is not a device
// address: host code reaches the array only through the address
// hipGetSymbolAddress gave for that device (scratch_base below).
constexpr uint64_t kNoAllocMaxText = 1ull << 33;  // bytes of text (8 GiB)
constexpr uint64_t kNoAllocTabWords = (sizeof(PfTab) + 255) / 256 * 32;  // whole 256-byte units
constexpr uint64_t kNoAllocStatusWords = 2 * ((kNoAllocMaxText + kPfTile - 1) / kPfTile + 1) + 1;
constexpr uint64_t kNoAllocWords = kNoAllocTabWords + kNoAllocStatusWords;
static_assert(kNoAllocMaxText == BT_NOALLOC_MAX_TEXT, "the header states the text bound");
static_assert(kNoAllocWords * 8 <= BT_NOALLOC_SCRATCH_BYTES, "the header states the size bound");
static __device__ __align__(256) uint64_t scratch[kNoAllocWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint64_t* g_scratch[kMaxDevices];  // per device: the array's address there, or null
bool g_scratch_looked_up[kMaxDevices];

// Look the array up on `device`, which must be current; once per device.
void scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_looked_up[device]) return;
  g_scratch_looked_up[device] = true;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess)
    g_scratch[device] = static_cast<uint64_t*>(p);
  else
    (void)hipGetLastError();  // reported by the entry point as BT_E_DEVICE
}

uint64_t* scratch_base(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch[device];
}
}  // namespace

// ------------------------------------------------------------------ context

struct KStat {
  uint64_t launches = 0;
  double ms = 0, bytes = 0, units = 0;
};

struct PendingEv {
  std::string name;
  hipEvent_t a, b;
  double bytes, units;
  const uint64_t* d_units;
  double bytes_per_unit;
  uint64_t wlen;  // window length of a scan launch (0 otherwise)
};

// One phase of a profiled build: step, block length, phase, blocks, then the
// device counters (keys, candidates, windows, verified, collisions).
struct PhaseRec {
  uint64_t v[9];
};

// One timed launch, in launch order.
struct LaunchRec {
  std::string name;
  uint64_t wlen;
  double units, ms, bytes;
};
constexpr size_t kLaunchLogMax = 1 << 16;

struct bt_ctx {
  int dev = 0;
  hipStream_t stream = nullptr;
  std::shared_ptr<Pool> pool;
  std::string err = "no error";
  bool profile = false;
  std::map<std::string, KStat> stats;
  std::vector<LaunchRec> launches;  // at most kLaunchLogMax, oldest first
  std::vector<PhaseRec> phases;     // at most kLaunchLogMax
  bt_tuning tune{1, 5, 0, 24};      // see bt_ctx_set_tuning
  std::vector<PendingEv> pending;
  std::vector<hipEvent_t> ev_free;
  uint64_t* h_small = nullptr;  // pinned host words for count read-back
  size_t h_small_words = 0;
  PfTab* h_tab = nullptr;       // pinned staging for the prefix-scan tables
  // pinned staging of host-to-device uploads: a bump region that is reused
  // only after the stream has been synchronized (every earlier upload is done)
  uint64_t* h_stage = nullptr;
  size_t h_stage_words = 0, h_stage_used = 0;
};

// Device-resident storage shared by the trees of one build.
struct Storage {
  std::shared_ptr<Pool> pool;
  std::vector<void*> bufs;
  uint64_t bytes = 0;
  ~Storage() {
    for (void* p : bufs) pool->put(p);
  }
  template <typename T>
  T* add(Buf<T>&& b, uint64_t n) {
    bytes += n * sizeof(T);
    T* p = b.release();
    bufs.push_back(p);
    return p;
  }
};

struct TreeLevel {
  uint64_t b = 0, c = 0, u = 0;
  const uint64_t* words = nullptr;  // ceil(c/64)
  const uint64_t* wrank = nullptr;  // marks before each word
  const uint64_t* pb = nullptr;     // u
  const uint64_t* po = nullptr;     // u
  // rank/select support (the forms are described in rank.hip)
  const uint32_t* acnt = nullptr;   // c * S absolute counts, or null:
  const uint8_t* qc = nullptr;      // c * S relative counts, qw bytes each
  const uint8_t* pc = nullptr;      // u * S pointer counts, pw bytes each
  const uint32_t* msel = nullptr;   // index of each marked block
  const uint64_t* st = nullptr;     // c
  uint32_t qw = 0, pw = 0;
};

struct bt_tree {
  std::shared_ptr<Storage> store;
  int dev = 0;
  uint64_t n = 0, b1 = 0;
  uint32_t tau = 0, leaf = 0, h = 0;
  std::vector<TreeLevel> lv;
  const uint8_t* leaves = nullptr;
  uint64_t leaf_bytes = 0;
  QLevel* d_levels = nullptr;  // device copy of the level table for queries
  uint64_t dev_bytes = 0;
  uint64_t rank_bytes = 0;  // of dev_bytes, the rank/select support's
  // rank/select support
  bool has_rank = false;
  const int16_t* sym = nullptr;   // 256 entries
  uint32_t S = 0;
  const uint64_t* total = nullptr;
  uint64_t tstart = 0;
};

// ------------------------------------------------------------------ helpers

namespace {

struct Fail {
  int code;
};

#define HIPCHK(ctx, expr)                                                              \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);                  \
      throw Fail{BT_E_DEVICE};                                                         \
    }                                                                                  \
  } while (0)

template <typename T>
Buf<T> alloc(bt_ctx* ctx, uint64_t n) {
  Buf<T> b;
  b.pool = ctx->pool;
  b.n = n;
  b.p = static_cast<T*>(ctx->pool->get((n ? n : 1) * sizeof(T)));
  if (!b.p) {
    ctx->err = "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed";
    throw Fail{BT_E_NOMEM};
  }
  return b;
}

uint64_t host_mul61(uint64_t a, uint64_t b) {
  const unsigned __int128 p = (unsigned __int128)a * b;
  uint64_t r = (uint64_t)(p & kP61Host) + (uint64_t)(p >> 61);
  return r >= kP61Host ? r - kP61Host : r;
}
uint64_t host_pow61(uint64_t x, uint64_t e) {
  uint64_t r = 1;
  while (e) {
    if (e & 1) r = host_mul61(r, x);
    x = host_mul61(x, x);
    e >>= 1;
  }
  return r;
}
uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Base x in [2^8, 2^61 - 1) from the seed.
uint64_t base_from_seed(uint64_t seed) {
  uint64_t s = seed;
  const uint64_t r = splitmix64(s);
  return 256 + r % (kP61Host - 1 - 256);
}

// Odd base of the 32-bit pre-filter hash (an even base would make the hash of
// a long window depend on its last 32 bytes only).
uint32_t base32_from_seed(uint64_t seed) {
  uint64_t s = seed ^ 0x32B17ull;
  splitmix64(s);
  uint32_t x = (uint32_t)(splitmix64(s) >> 17) | 1u;
  return x == 1u ? 0x9E3779B1u : x;
}

uint32_t host_pow32(uint32_t x, uint64_t e) {
  uint32_t r = 1;
  while (e) {
    if (e & 1) r *= x;
    x *= x;
    e >>= 1;
  }
  return r;
}

// x^-1 mod 2^32 for odd x: Newton's iteration y <- y (2 - x y) doubles the
// number of correct low bits, and y = x is right to 3 bits (x x = 1 mod 8).
uint32_t host_inv32(uint32_t x) {
  uint32_t y = x;
  for (int k = 0; k < 4; ++k) y *= 2u - x * y;
  return y;
}

// Tables of the prefix scan: g61[j-1][b] = b x^j (j = 1..7), t[k] = x^(64 k),
// xt[k] = x^(tile k), c[c] = x^(16 c), for both bases.
void fill_tab(PfTab* tb, uint64_t x, uint32_t x32) {
  uint64_t xj = 1;
  uint32_t yj = 1;
  for (int j = 1; j <= 7; ++j) {
    xj = host_mul61(xj, x);
    yj *= x32;
    for (int b = 0; b < 256; ++b) tb->g61[j - 1][b] = host_mul61(xj, (uint64_t)b);
  }
  tb->x1_61 = x;
  tb->x8_61 = host_mul61(xj, x);
  tb->x1_32 = x32;
  tb->x8_32 = yj * x32;
  const uint64_t x64 = host_pow61(x, 64);
  const uint32_t y64 = host_pow32(x32, 64);
  tb->t61[0] = 1;
  tb->t32[0] = 1;
  for (int k = 1; k <= kPfThreads; ++k) {
    tb->t61[k] = host_mul61(tb->t61[k - 1], x64);
    tb->t32[k] = tb->t32[k - 1] * y64;
  }
  const uint64_t xt = host_pow61(x, kPfTile);
  const uint32_t yt = host_pow32(x32, kPfTile);
  tb->xt61[0] = 1;
  tb->xt32[0] = 1;
  for (int k = 1; k <= 64; ++k) {
    tb->xt61[k] = host_mul61(tb->xt61[k - 1], xt);
    tb->xt32[k] = tb->xt32[k - 1] * yt;
  }
  for (int c = 0; c < 4; ++c) {
    tb->c61[c] = host_pow61(x, 16 * c);
    tb->c32[c] = host_pow32(x32, 16 * c);
  }
}

hipEvent_t get_event(bt_ctx* ctx) {
  if (!ctx->ev_free.empty()) {
    hipEvent_t e = ctx->ev_free.back();
    ctx->ev_free.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(ctx, hipEventCreate(&e));
  return e;
}

// Time one launch (a callable returning hipError_t) when profiling is on.
// `bytes`/`units` are the launch's algorithmic bytes and work units; when
// d_units is given, the unit count is read from device memory after the next
// synchronisation and bytes = units * bytes_per_unit.
template <typename F>
void timed(bt_ctx* ctx, const char* name, double bytes, double units, const uint64_t* d_units,
           double bytes_per_unit, F&& f, uint64_t wlen = 0) {
  if (!ctx->profile) {
    HIPCHK(ctx, f());
    return;
  }
  hipEvent_t a = get_event(ctx), b = get_event(ctx);
  HIPCHK(ctx, hipEventRecord(a, ctx->stream));
  HIPCHK(ctx, f());
  HIPCHK(ctx, hipEventRecord(b, ctx->stream));
  ctx->pending.push_back({name, a, b, bytes, units, d_units, bytes_per_unit, wlen});
}

// Folds finished timed launches into the statistics.  A launch whose unit
// count lives on the device (d_units) waits until the caller passes a host
// copy of the region holding it ([dbase, dbase + len) -> hbase); the build reads
// that region once at its end instead of one blocking copy per launch.
void collect_events(bt_ctx* ctx, const uint64_t* dbase = nullptr, const uint64_t* hbase = nullptr,
                    uint64_t len = 0) {
  std::vector<PendingEv> keep;
  for (auto& p : ctx->pending) {
    double units = p.units, bytes = p.bytes;
    if (p.d_units) {
      if (!(dbase && p.d_units >= dbase && p.d_units < dbase + len)) {
        keep.push_back(p);
        continue;
      }
      units = (double)hbase[p.d_units - dbase];
      bytes = units * p.bytes_per_unit;
    }
    float ms = 0;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      KStat& s = ctx->stats[p.name];
      s.launches++;
      s.ms += ms;
      s.bytes += bytes;
      s.units += units;
      if (ctx->launches.size() < kLaunchLogMax)
        ctx->launches.push_back({p.name, p.wlen, units, (double)ms, bytes});
    }
    ctx->ev_free.push_back(p.a);
    ctx->ev_free.push_back(p.b);
  }
  ctx->pending.swap(keep);
}

uint64_t* small_host(bt_ctx* ctx, size_t words) {
  if (words > ctx->h_small_words) {
    if (ctx->h_small) (void)hipHostFree(ctx->h_small);
    ctx->h_small = nullptr;
    size_t w = std::max<size_t>(words, 64);
    HIPCHK(ctx, hipHostMalloc((void**)&ctx->h_small, w * 8, hipHostMallocDefault));
    ctx->h_small_words = w;
  }
  return ctx->h_small;
}

// Pinned staging for an upload of `words` u64 (see bt_ctx::h_stage).
uint64_t* stage_host(bt_ctx* ctx, size_t words) {
  if (ctx->h_stage_used + words > ctx->h_stage_words) {
    // queued uploads may still read the region: let them finish first
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->h_stage_used = 0;
    if (words > ctx->h_stage_words) {
      if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
      ctx->h_stage = nullptr;
      ctx->h_stage_words = 0;
      const size_t w = std::max<size_t>({words, 2 * ctx->h_stage_words, 1 << 16});
      HIPCHK(ctx, hipHostMalloc((void**)&ctx->h_stage, w * 8, hipHostMallocDefault));
      ctx->h_stage_words = w;
    }
  }
  uint64_t* p = ctx->h_stage + ctx->h_stage_used;
  ctx->h_stage_used += words;
  return p;
}

// Read `words` u64 from device (stream-ordered, then synchronise).
void read_words(bt_ctx* ctx, std::vector<std::pair<const uint64_t*, uint64_t>> src,
                std::vector<uint64_t>& out) {
  uint64_t tot = 0;
  for (auto& s : src) tot += s.second;
  uint64_t* h = small_host(ctx, tot);
  uint64_t o = 0;
  for (auto& s : src) {
    if (s.second)
      HIPCHK(ctx, hipMemcpyAsync(h + o, s.first, s.second * 8, hipMemcpyDeviceToHost, ctx->stream));
    o += s.second;
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->h_stage_used = 0;  // every queued upload has completed
  collect_events(ctx);
  out.assign(h, h + tot);
}

template <typename T>
void upload(bt_ctx* ctx, T* d, const T* h, uint64_t n) {
  if (!n) return;
  // stage through pinned memory: the copy is stream-ordered, and the host
  // does not wait for it
  const uint64_t words = (n * sizeof(T) + 7) / 8;
  uint64_t* st = stage_host(ctx, words);
  std::memcpy(st, h, n * sizeof(T));
  HIPCHK(ctx, hipMemcpyAsync(d, st, n * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
}

struct Plan {
  uint64_t b1;
  uint32_t h;
};

int plan_text(uint64_t n, const bt_params& p, Plan* out) {
  uint64_t b = p.leaf_len;
  uint32_t k = 0;
  if (p.root_block_len) {
    while (b < p.root_block_len) {
      if (b > UINT64_MAX / p.tau) return BT_E_INVAL;
      b *= p.tau;
      ++k;
    }
    if (b != p.root_block_len) return BT_E_INVAL;
  } else {
    const uint64_t s = p.s_hint ? p.s_hint : 1;
    const uint64_t lim = n / s;
    while (b <= lim / p.tau) {
      b *= p.tau;
      ++k;
    }
  }
  out->b1 = b;
  out->h = k + 1;
  return BT_OK;
}

uint64_t pow2_at_least(uint64_t v) {
  uint64_t r = 1;
  while (r < v) r <<= 1;
  return r;
}


// Per-text, per-level bookkeeping collected on the host.
struct TextLevelRec {
  uint64_t b, c, u, word_off, ptr_off, first;
};

struct LevelBufs {
  uint64_t* words = nullptr;
  uint64_t* wrank = nullptr;
  uint64_t* pb = nullptr;
  uint64_t* po = nullptr;
  // rank/select support of the step: absolute counts of every block (acnt), or
  // relative ones (qc) plus absolute rows for the texts whose tree starts here
  // (aroot, text t's rows from root_row[t])
  uint32_t* acnt = nullptr;
  uint8_t* qc = nullptr;
  uint32_t* aroot = nullptr;
  std::vector<uint64_t> root_row;
  uint8_t* pc = nullptr;
  uint32_t* msel = nullptr;
  uint64_t* st = nullptr;
  uint32_t qw = 0, pw = 0;
};

int build_many(bt_ctx* ctx, const uint8_t* d_base, const std::vector<uint64_t>& offs,
               uint32_t sigma, const bt_params& prm, bt_tree** outs) {
  const uint32_t T = (uint32_t)(offs.size() - 1);
  if (prm.tau < 2 || prm.leaf_len == 0 || sigma < 1 || sigma > 256) {
    ctx->err = "invalid parameters (tau >= 2, leaf_len >= 1, sigma in 1..256)";
    return BT_E_INVAL;
  }
  for (uint32_t t = 0; t < T; ++t)
    if (offs[t + 1] < offs[t]) {
      ctx->err = "text offsets must be non-decreasing";
      return BT_E_INVAL;
    }
  std::vector<Plan> plan(T);
  uint32_t H = 1;
  for (uint32_t t = 0; t < T; ++t) {
    if (plan_text(offs[t + 1] - offs[t], prm, &plan[t]) != BT_OK) {
      ctx->err = "root_block_len must equal leaf_len * tau^k";
      return BT_E_INVAL;
    }
    H = std::max(H, plan[t].h);
  }
  if (T == 0) return BT_OK;
  if (!d_base && offs[T] > offs[0]) {
    ctx->err = "null text pointer";
    return BT_E_INVAL;
  }
  for (uint32_t k = 1; k < H; ++k)
    if ((uint64_t)prm.leaf_len > UINT64_MAX / 2 / prm.tau) {
      ctx->err = "block length overflows";
      return BT_E_INVAL;
    }

  HIPCHK(ctx, hipSetDevice(ctx->dev));
  hipStream_t s = ctx->stream;
  const uint64_t o0 = offs[0], N = offs[T] - offs[0];
  const uint64_t x = base_from_seed(prm.hash_seed);
  const uint64_t fpmask = (prm.debug_flags & BT_DBG_WEAK_HASH) ? 0xFFFull : ~0ull;
  const bool has_salt = T > 1;

  // ---- texts
  std::vector<uint64_t> h_tx(3 * (size_t)T), h_n(T);
  uint64_t sm = prm.hash_seed ^ 0x5A17ull;
  for (uint32_t t = 0; t < T; ++t) {
    h_tx[t] = offs[t];
    h_tx[T + t] = offs[t + 1];
    h_tx[2 * T + t] = has_salt ? splitmix64(sm) % kP61Host : 0;
    h_n[t] = offs[t + 1] - offs[t];
  }
  Buf<uint64_t> d_tx = alloc<uint64_t>(ctx, 3 * (uint64_t)T);
  upload(ctx, d_tx.p, h_tx.data(), 3 * (uint64_t)T);
  TextsDev tx{T, d_tx.p, d_tx.p + T, d_tx.p + 2 * T};

  // ---- which byte values occur (read back after the prefix scan is queued)
  Buf<uint64_t> d_seen = alloc<uint64_t>(ctx, 4);
  HIPCHK(ctx, launch_fill_u64(d_seen.p, 0, 4, s));
  HIPCHK(ctx, launch_byte_presence(d_base + o0, N, reinterpret_cast<uint32_t*>(d_seen.p), s));

  // ---- step a2: prefix fingerprints of the concatenation, once, and in the
  // same pass the 32-bit pre-filter hashes (same indexing).  A memory-lean
  // build keeps one fingerprint in 16 (0.5 instead of 8 bytes per text byte)
  // and forms the others where a fingerprint is needed: keys, queued
  // candidates and retries.  Only the queued scan takes candidates that way.
  // It samples the 32-bit hashes too (0.25 instead of 4 bytes per text byte):
  // the scans roll them along consecutive windows.
  const bool can_sample = T <= (1u << 24) && offs[T] < (1ull << 40) &&
                          !(prm.debug_flags & BT_DBG_NO_QUEUE);
  const bool lean = (prm.flags & BT_LEAN) && can_sample;  // both kinds sampled
  const bool sample_p = lean;  // the fingerprints sampled
  // Other queued single-text builds keep the fingerprints every 4th position
  // beside the dense 32-bit hashes: 2 instead of 8 bytes per text byte to
  // write, and a candidate's fingerprint costs at most three Horner steps per
  // end (measured: 2 GiB DNA 159.6 -> 155.4 ms; the batch scan lost as much as
  // the prefix pass gained, so batches keep them dense).
  const bool quarter_p = !lean && can_sample && T == 1;
  const uint32_t x32 = base32_from_seed(prm.hash_seed);
  const uint64_t np = sample_p ? N / 16 + 1 : quarter_p ? N / 4 + 1 : N + 1,
                 nh = lean ? N / 16 + 1 : N + 1;
  Buf<uint64_t> d_P = alloc<uint64_t>(ctx, np);
  Buf<uint32_t> d_H = alloc<uint32_t>(ctx, nh);
  Buf<PfTab> d_tab = alloc<PfTab>(ctx, 1);
  fill_tab(ctx->h_tab, x, x32);
  HIPCHK(ctx, hipMemcpyAsync(d_tab.p, ctx->h_tab, sizeof(PfTab), hipMemcpyHostToDevice, s));
  Buf<uint64_t> d_status = alloc<uint64_t>(ctx, prefix_status_words(N));
  timed(ctx, "prefix_fp", (double)N + 8.0 * (double)np + 4.0 * (double)nh, (double)N, nullptr, 0,
        [&] { return launch_prefix(d_base + o0, N, d_P.p, sample_p, d_H.p, d_tab.p, d_status.p, s, lean,
                                   quarter_p); });
  // P[i] belongs to text position i (never read below o0); null when sampled
  const uint64_t* P = (sample_p || quarter_p) ? nullptr : d_P.p - o0;

  // ---- distinct byte values must not exceed sigma; dense symbols for rank/select
  std::vector<uint64_t> seen;
  read_words(ctx, {{d_seen.p, 4}}, seen);
  uint32_t S = 0;
  std::vector<int16_t> h_sym(256, -1);
  std::vector<uint8_t> h_byte_of;
  for (int ch = 0; ch < 256; ++ch)
    if ((seen[ch >> 6] >> (ch & 63)) & 1) {
      h_sym[ch] = (int16_t)S++;
      h_byte_of.push_back((uint8_t)ch);
    }
  if (S > sigma) {
    ctx->err = "the text has " + std::to_string(S) + " distinct byte values, more than sigma";
    return BT_E_INVAL;
  }
  const bool with_rank = (prm.flags & BT_WITH_RANK_SELECT) != 0;
  if (with_rank)
    for (uint32_t t = 0; t < T; ++t)
      if (h_n[t] >= (1ull << 32)) {
        ctx->err = "rank/select support needs texts shorter than 2^32 bytes";
        return BT_E_INVAL;
      }
  // H[i] belongs to text position i; null when sampled (Hs = d_H)
  const uint32_t* H32 = lean ? nullptr : d_H.p - o0;

  auto store = std::make_shared<Storage>();
  store->pool = ctx->pool;

  // ---- rank/select support: sampled count table and per-text counts
  RankCtx rc{};
  Buf<uint64_t> d_G, d_Rt;
  uint64_t* d_Rtot = nullptr;
  int16_t* d_sym = nullptr;
  if (with_rank && S) {
    Buf<int16_t> sym = alloc<int16_t>(ctx, 256);
    upload(ctx, sym.p, h_sym.data(), 256);
    Buf<uint8_t> byte_of = alloc<uint8_t>(ctx, S);
    upload(ctx, byte_of.p, h_byte_of.data(), S);
    const uint64_t K = (N + kRankQ - 1) / kRankQ;
    const uint64_t nblk = (K + 1023) / 1024;
    Buf<uint32_t> H = alloc<uint32_t>(ctx, std::max<uint64_t>(K, 1) * S);
    Buf<uint64_t> B = alloc<uint64_t>(ctx, std::max<uint64_t>(nblk, 1) * S);
    d_G = alloc<uint64_t>(ctx, (K + 1) * S);
    HIPCHK(ctx, launch_fill_u64(d_G.p, 0, S, s));
    HIPCHK(ctx, build_count_table(d_base, o0, N, sym.p, S, H.p, B.p, d_G.p, s));
    rc = RankCtx{d_base, o0, d_G.p, S, byte_of.p};
    d_Rt = alloc<uint64_t>(ctx, (uint64_t)T * S);
    Buf<uint64_t> Rtot = alloc<uint64_t>(ctx, (uint64_t)T * S);
    HIPCHK(ctx, launch_text_rank_counts(rc, tx, d_Rt.p, Rtot.p, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    d_Rtot = store->add(std::move(Rtot), (uint64_t)T * S);
    d_sym = store->add(std::move(sym), 256);
    store->add(std::move(byte_of), S);
  }
  const bool rank_on = with_rank && S;
  const bool prune = (prm.flags & BT_PRUNE) != 0;

  // ---- outputs
  // per text, its levels (a text whose tree is shorter enters at a later step)
  std::vector<std::vector<TextLevelRec>> rec(T);
  for (uint32_t t = 0; t < T; ++t) rec[t].resize(plan[t].h);
  std::vector<LevelBufs> lbufs(H);  // by step
  uint8_t* leaves = nullptr;
  std::vector<uint64_t> leaf_off(T, 0), leaf_bytes(T, 0);
  Buf<uint64_t> d_err = alloc<uint64_t>(ctx, 1);
  HIPCHK(ctx, launch_fill_u64(d_err.p, 0, 1, s));
  Buf<uint64_t> wstats = alloc<uint64_t>(ctx, 2 * (uint64_t)H + 2);
  // per (step, phase) device counters while profiling (PhaseArgs.pc)
  Buf<uint64_t> pstats;
  std::vector<std::array<uint64_t, 4>> phase_host;  // step, b, phase, blocks
  if (ctx->profile) {
    pstats = alloc<uint64_t>(ctx, 2 * (uint64_t)H * kPcWords);
    HIPCHK(ctx, launch_fill_u64(pstats.p, 0, 2 * (uint64_t)H * kPcWords, s));
  }

  // ---- level state
  uint64_t c = 0;
  Buf<uint64_t> st;
  Buf<uint32_t> text;
  // scan entries of the current level (from the previous level's split; see
  // "scan segments" in level.hip); E_ent = 0 means "one entry per run"
  uint64_t E_ent = 0;
  Buf<uint64_t> ent_a, ent_e, ent_child;
  Buf<uint8_t> ent_f;
  bool have_entries = false;
  std::vector<uint64_t> h_tcount(T, 0), h_tfirst(T + 1, 0);
  Buf<uint64_t> d_tcount = alloc<uint64_t>(ctx, T + 1), d_tfirst = alloc<uint64_t>(ctx, T + 1);
  Buf<uint64_t> scan_tmp;
  auto scan = [&](uint64_t* a, uint64_t n) {
    const uint64_t w = scan_tmp_words(n);
    if (!scan_tmp.p || scan_tmp.n < w) scan_tmp = alloc<uint64_t>(ctx, std::max<uint64_t>(w, 1024));
    HIPCHK(ctx, scan_excl_u64(a, n, scan_tmp.p, s));
  };
  const auto b_at = [&](uint32_t step) {
    uint64_t b = prm.leaf_len;
    for (uint32_t k = step + 1; k < H; ++k) b *= prm.tau;
    return b;
  };
  // texts whose level 1 is the level of `step`, and their level-1 block counts
  auto entering = [&](uint32_t step, std::vector<uint32_t>& ids, std::vector<uint64_t>& cnt,
                      uint64_t b) {
    ids.clear();
    cnt.assign(T, 0);
    for (uint32_t t = 0; t < T; ++t)
      if (H - plan[t].h == step) {
        ids.push_back(t);
        cnt[t] = (h_n[t] + b - 1) / b;
      }
  };
  const auto check_runs = [&](uint64_t device_R, uint64_t R) {
    if (device_R != R) {
      ctx->err = "internal: predicted run count differs from the device's";
      throw Fail{BT_E_INTERNAL};
    }
  };
  // ---- rank/select counts of a level from its absolute counts A: kept as they
  // are where relative counts would need 32 bits, else narrowed to counts
  // inside the parent (at most (tau - 1) b) with absolute rows for the texts
  // whose tree starts at this step.  Also keeps the block starts (select).
  uint64_t rank_bytes = 0;
  auto rank_counts = [&](uint32_t step, uint64_t b, uint64_t c, const uint64_t* st,
                         const uint32_t* text, const uint64_t* d_tf,
                         const std::vector<uint64_t>& tcount, const std::vector<uint64_t>& tfirst,
                         Buf<uint32_t>& A, LevelBufs& LB) {
    Buf<uint64_t> stc = alloc<uint64_t>(ctx, c);
    if (c) HIPCHK(ctx, hipMemcpyAsync(stc.p, st, c * 8, hipMemcpyDeviceToDevice, s));
    LB.st = store->add(std::move(stc), c);
    rank_bytes += 8 * c;
    LB.qw = counter_width((uint64_t)(prm.tau - 1) * b);
    if (LB.qw == 4) {
      LB.acnt = store->add(std::move(A), c * S);
      rank_bytes += 4 * c * S;
      return;
    }
    Buf<uint8_t> q = alloc<uint8_t>(ctx, c * S * LB.qw);
    HIPCHK(ctx, launch_relative_counts(A.p, c, S, text, d_tf, prm.tau, q.p, LB.qw, s));
    LB.qc = store->add(std::move(q), c * S * LB.qw);
    rank_bytes += (uint64_t)LB.qw * c * S;
    std::vector<uint64_t> ent;
    uint64_t rows = 0;
    LB.root_row.assign(T, ~0ull);
    for (uint32_t t = 0; t < T; ++t)
      if (H - plan[t].h == step && tcount[t]) {
        ent.insert(ent.end(), {tfirst[t], tcount[t], rows});
        LB.root_row[t] = rows;
        rows += tcount[t];
      }
    if (!rows) return;
    const uint32_t E = (uint32_t)(ent.size() / 3);
    Buf<uint64_t> d_ent = alloc<uint64_t>(ctx, ent.size());
    upload(ctx, d_ent.p, ent.data(), ent.size());
    Buf<uint32_t> ar = alloc<uint32_t>(ctx, rows * S);
    HIPCHK(ctx, launch_root_rows(A.p, S, d_ent.p, E, ar.p, s));
    LB.aroot = store->add(std::move(ar), rows * S);
    rank_bytes += 4 * rows * S;
  };
  // ---- tree storage of an internal level: marks packed per text (with their
  // ranks), the pointers (by unmarked rank; the buffers move into the storage)
  // and the rank/select counters.  uoff: exclusive scan of the unmarked flags.
  auto store_level = [&](uint32_t step, uint64_t b, uint64_t c, const uint64_t* st,
                         const uint32_t* text, const uint8_t* marked, const uint64_t* uoff,
                         Buf<uint64_t>& spb, Buf<uint64_t>& spo, uint64_t u,
                         const std::vector<uint64_t>& tcount, const std::vector<uint64_t>& tfirst,
                         const std::vector<uint64_t>& tu, const uint64_t* d_tf,
                         const uint64_t* d_tc) {
    std::vector<uint64_t> h_woff(T + 1, 0), h_poff(T + 1, 0);
    for (uint32_t t = 0; t < T; ++t) {
      h_woff[t + 1] = h_woff[t] + (tcount[t] + 63) / 64;
      h_poff[t + 1] = h_poff[t] + tu[t];
    }
    const uint64_t nwords = h_woff[T];
    Buf<uint64_t> d_woff = alloc<uint64_t>(ctx, T + 1);
    upload(ctx, d_woff.p, h_woff.data(), T + 1);
    Buf<uint64_t> words = alloc<uint64_t>(ctx, nwords), wrank = alloc<uint64_t>(ctx, nwords + 1);
    Buf<uint64_t> wtmp = alloc<uint64_t>(ctx, nwords + 1);
    HIPCHK(ctx, launch_pack_marks(marked, T, d_tf, d_tc, d_woff.p, nwords, words.p, s));
    HIPCHK(ctx, launch_word_pop(words.p, nwords, wtmp.p, s));
    scan(wtmp.p, nwords);
    HIPCHK(ctx, launch_word_rank(wtmp.p, T, d_woff.p, nwords, wrank.p, s));
    LevelBufs LB;
    LB.words = store->add(std::move(words), nwords);
    LB.wrank = store->add(std::move(wrank), nwords + 1);
    LB.pb = store->add(std::move(spb), u);
    LB.po = store->add(std::move(spo), u);
    if (rank_on) {
      Buf<uint32_t> A = alloc<uint32_t>(ctx, c * S);
      HIPCHK(ctx, launch_block_rank_counts(rc, st, text, c, d_Rt.p, A.p, s));
      // pointer counts: below b (the pointer arrays now belong to the storage)
      LB.pw = counter_width(b ? b - 1 : 0);
      Buf<uint8_t> pc = alloc<uint8_t>(ctx, u * S * LB.pw);
      HIPCHK(ctx, launch_pointer_rank_counts(rc, st, text, marked, c, uoff, d_tf, LB.pb, LB.po,
                                             d_Rt.p, A.p, pc.p, LB.pw, s));
      LB.pc = store->add(std::move(pc), u * S * LB.pw);
      Buf<uint32_t> msel = alloc<uint32_t>(ctx, c - u);
      HIPCHK(ctx, launch_marked_index(marked, uoff, c, text, d_tf, msel.p, s));
      LB.msel = store->add(std::move(msel), c - u);
      rank_bytes += (uint64_t)LB.pw * u * S + 4 * (c - u);
      rank_counts(step, b, c, st, text, d_tf, tcount, tfirst, A, LB);
    }
    lbufs[step] = std::move(LB);
    for (uint32_t t = 0; t < T; ++t)
      if (H - plan[t].h <= step)
        rec[t][step - (H - plan[t].h)] = {b, tcount[t], tu[t], h_woff[t], h_poff[t], tfirst[t]};
  };
  // ---- tree storage of the leaf level: block j's bytes at j*b (only a text's
  // last block is short, and it ends the text's region).  When runs_at is given,
  // the device's run count there is checked against R in the same read-back.
  auto store_leaf_level = [&](uint32_t step, uint64_t b, uint64_t c, const uint64_t* st,
                              const uint32_t* text, const std::vector<uint64_t>& tcount,
                              const std::vector<uint64_t>& tfirst, const uint64_t* d_tf,
                              const uint64_t* d_tc, const uint64_t* runs_at, uint64_t R) {
    LevelDev lvl{c, b, st, text, nullptr, 0, nullptr, nullptr, nullptr};
    Buf<uint8_t> lb = alloc<uint8_t>(ctx, c * b);
    HIPCHK(ctx, launch_leaves(d_base, lvl, tx, lb.p, s));
    leaves = store->add(std::move(lb), c * b);
    LevelBufs LL;
    if (rank_on) {
      Buf<uint32_t> A = alloc<uint32_t>(ctx, c * S);
      HIPCHK(ctx, launch_block_rank_counts(rc, st, text, c, d_Rt.p, A.p, s));
      rank_counts(step, b, c, st, text, d_tf, tcount, tfirst, A, LL);
    }
    lbufs[step] = std::move(LL);
    Buf<uint64_t> d_last = alloc<uint64_t>(ctx, T);
    HIPCHK(ctx, launch_last_block_len(lvl, tx, d_tf, d_tc, d_last.p, s));
    std::vector<uint64_t> last;
    read_words(ctx, {{d_last.p, T}, {runs_at, runs_at ? 1u : 0u}}, last);
    if (runs_at) check_runs(last[T], R);
    for (uint32_t t = 0; t < T; ++t) {
      leaf_off[t] = tfirst[t] * b;
      leaf_bytes[t] = tcount[t] ? (tcount[t] - 1) * b + last[t] : 0;
      rec[t][plan[t].h - 1] = {b, tcount[t], 0, 0, 0, tfirst[t]};
    }
  };

  // What the optional pruning pass needs of each level, kept from the build:
  // the built (unpruned) layout, the marks, every block's leftmost occurrence
  // on its level, and where each block's children start.
  struct PruneLevel {
    uint64_t b = 0, c = 0;
    Buf<uint64_t> st, lm, cs, tfirst, tcount;
    Buf<uint32_t> text, run;
    Buf<uint8_t> marked;
    std::vector<uint64_t> h_tcount, h_tfirst;
  };
  std::vector<PruneLevel> pl(prune ? H : 0);

  {
    const uint64_t b0 = b_at(0);
    std::vector<uint32_t> ids;
    std::vector<uint64_t> cnt;
    entering(0, ids, cnt, b0);
    for (uint32_t t = 0; t < T; ++t) h_tfirst[t + 1] = h_tfirst[t] + cnt[t];
    c = h_tfirst[T];
    h_tcount = cnt;
    upload(ctx, d_tcount.p, h_tcount.data(), T);
    upload(ctx, d_tfirst.p, h_tfirst.data(), T + 1);
    st = alloc<uint64_t>(ctx, c);
    text = alloc<uint32_t>(ctx, c);
    Buf<uint32_t> d_ids = alloc<uint32_t>(ctx, ids.size());
    upload(ctx, d_ids.p, ids.data(), ids.size());
    HIPCHK(ctx, launch_write_entering(d_ids.p, (uint32_t)ids.size(), tx, b0, d_tfirst.p, st.p,
                                      text.p, s));
  }

  // Runs of the first level: one per non-empty text that enters there.  Each
  // later level's count comes from the level before it (k_mark_facts), so no
  // level waits for its own count; the device's count is checked against it
  // at the level's first read-back.
  uint64_t R_pred = 0;
  for (uint32_t t = 0; t < T; ++t) R_pred += h_tcount[t] ? 1 : 0;

  for (uint32_t step = 0; step < H; ++step) {
    const uint64_t b = b_at(step);
    const bool leaf_step = (step == H - 1);

    // runs of this level (maximal sequences of consecutive blocks of one text)
    Buf<uint64_t> roff = alloc<uint64_t>(ctx, c + 1);
    Buf<uint32_t> run = alloc<uint32_t>(ctx, c);
    HIPCHK(ctx, launch_run_flags(st.p, text.p, c, b, roff.p, s));
    scan(roff.p, c);
    const uint64_t R = R_pred;
    // sized by c, which bounds any run count: the run table is indexed by the
    // device's own count, which is checked against R only later
    Buf<uint64_t> rs = alloc<uint64_t>(ctx, c), re = alloc<uint64_t>(ctx, c);
    Buf<uint32_t> rtext = alloc<uint32_t>(ctx, c);
    HIPCHK(ctx, launch_run_table(st.p, text.p, c, b, tx, roff.p, run.p, rs.p, re.p, rtext.p, s));
    LevelDev lv{c, b, st.p, text.p, run.p, R, rs.p, re.p, rtext.p};
    Buf<uint32_t> ent_run;
    if (!leaf_step) {
      if (!have_entries) {
        E_ent = R;
        ent_a = alloc<uint64_t>(ctx, R);
        ent_e = alloc<uint64_t>(ctx, R);
        ent_f = alloc<uint8_t>(ctx, R);
        ent_run = alloc<uint32_t>(ctx, R);
        HIPCHK(ctx, launch_entries_from_runs(lv, ent_a.p, ent_e.p, ent_f.p, ent_run.p, s));
      } else {
        ent_run = alloc<uint32_t>(ctx, E_ent);
        HIPCHK(ctx, launch_entry_runs(ent_child.p, E_ent, run.p, ent_run.p, s));
      }
    }

    if (leaf_step) {
      if (!prune) {
        store_leaf_level(step, b, c, st.p, text.p, h_tcount, h_tfirst, d_tfirst.p, d_tcount.p,
                         roff.p + c, R);
      } else {
        std::vector<uint64_t> rr;
        read_words(ctx, {{roff.p + c, 1}}, rr);
        check_runs(rr[0], R);
        PruneLevel& K = pl[step];
        K.b = b;
        K.c = c;
        K.st = std::move(st);
        K.text = std::move(text);
        K.tfirst = std::move(d_tfirst);
        K.tcount = std::move(d_tcount);
        K.h_tcount = h_tcount;
        K.h_tfirst = h_tfirst;
      }
      break;
    }

    // a text whose final block is present and short has odd-length keys
    bool has_odd = false;
    for (uint32_t t = 0; t < T; ++t)
      if (h_tcount[t] && (h_n[t] % b) != 0) has_odd = true;

    const uint64_t cap = std::max<uint64_t>(1024, pow2_at_least(c << ctx->tune.table_load_log2));
    Buf<Slot> tab = alloc<Slot>(ctx, cap);
    Buf<uint64_t> kfp = alloc<uint64_t>(ctx, c), klen = alloc<uint64_t>(ctx, c),
                  klm = alloc<uint64_t>(ctx, c);
    Buf<uint32_t> kslot = alloc<uint32_t>(ctx, c);
    Buf<uint64_t> oddb = alloc<uint64_t>(ctx, 7 * (uint64_t)T);
    Buf<uint64_t> woff = alloc<uint64_t>(ctx, E_ent + 1);
    Buf<uint64_t> seg_ws = alloc<uint64_t>(ctx, E_ent), seg_re = alloc<uint64_t>(ctx, E_ent);
    Buf<uint32_t> seg_text = alloc<uint32_t>(ctx, E_ent);
    SegDev sg{E_ent, ent_a.p, ent_e.p, ent_f.p, ent_run.p, seg_ws.p, seg_re.p, seg_text.p};
    Buf<uint8_t> facts = alloc<uint8_t>(ctx, c);
    Buf<uint32_t> vlist = alloc<uint32_t>(ctx, c), vmis = alloc<uint32_t>(ctx, c),
                  rlist = alloc<uint32_t>(ctx, c);
    Buf<uint64_t> vbest = alloc<uint64_t>(ctx, c), rlb = alloc<uint64_t>(ctx, c),
                  vcnt = alloc<uint64_t>(ctx, 2);
    Buf<uint8_t> marked = alloc<uint8_t>(ctx, c);
    // LDS key filter of up to 2^19 bits, sized per phase from the key count
    Buf<uint32_t> filt = alloc<uint32_t>(ctx, (1ull << 19) / 32);
    // second key filter (global memory, at most 2^24 bits = 2 MiB: stays in L2)
    Buf<uint32_t> filt2 = alloc<uint32_t>(ctx, (1ull << ctx->tune.filter2_max_log2) / 32);
    int scan_mode = 1;
    uint32_t fbits = 12;
    VerifyBufs vb{vlist.p, vbest.p, vmis.p, rlist.p, rlb.p, vcnt.p};

    PhaseArgs a{};
    a.T = d_base;
    a.P = P;
    a.Ps = (sample_p || quarter_p) ? d_P.p : nullptr;
    a.pshift = quarter_p ? 2 : 4;
    a.pbase = o0;
    a.pend = offs[T];
    a.P32 = H32;
    a.Hs = lean ? d_H.p : nullptr;
    a.x32inv = host_inv32(x32);
    a.tx = tx;
    a.lv = lv;
    a.k = KeysDev{kfp.p, klen.p, kslot.p, klm.p};
    a.odd = OddDev{oddb.p,         oddb.p + T,     oddb.p + 2 * T, oddb.p + 3 * T,
                   oddb.p + 4 * T, oddb.p + 5 * T, oddb.p + 6 * T};
    a.x32 = x32;
    a.tab = TableDev{tab.p, cap - 1};
    a.x = x;
    a.fpmask = fpmask;
    a.marked = marked.p;
    a.filt = filt.p;
    a.filt2 = filt2.p;
    // parent facts per block: keys inside a parent region that occurs earlier
    // are known copies and stay out of the table
    Buf<uint8_t> cflag;
    if (have_entries && c) {
      cflag = alloc<uint8_t>(ctx, c);
      HIPCHK(ctx, launch_fill_u8(cflag.p, 0, c, s));
      HIPCHK(ctx, launch_child_flags(sg, b, ent_child.p, cflag.p, s));
      a.cflag = cflag.p;
    }
    a.exact_all = prune ? 1 : 0;

    // Phase-2 segments come from this level's blocks and pair facts.
    Buf<uint64_t> bwc = alloc<uint64_t>(ctx, c + 1), bhd = alloc<uint64_t>(ctx, c + 1);
    Buf<uint64_t> bws = alloc<uint64_t>(ctx, c), bre = alloc<uint64_t>(ctx, c);
    Buf<uint64_t> bwoff = alloc<uint64_t>(ctx, c + 1);
    Buf<uint32_t> btext = alloc<uint32_t>(ctx, c);

    // Text-local filters (batches): per text, 2^wl 32-bit words with wl the
    // least >= 3 such that each of the text's blocks (a bound on its keys in
    // either phase) has a word.  One layout serves both phases.
    // A text whose filter is larger than LDS also gets a folded copy of LDS
    // size (tf_fold), built after the keys.
    Buf<uint64_t> tf_off, tf_fold_off, span_ctr;
    Buf<uint32_t> tf_words, tf_wl, tf_fold, tf_big;
    uint64_t tf_total = 0;
    uint32_t nbig = 0;
    if (has_salt && c && !(prm.debug_flags & (BT_DBG_SHARED_FILTERS | BT_DBG_SORT_PHASES))) {
      std::vector<uint64_t> h_off(T), h_foff(T, 0);
      std::vector<uint32_t> h_wl(T), h_big;
      const uint32_t tf_lds = kTextFilterLdsLog2;
      for (uint32_t t = 0; t < T; ++t) {
        uint32_t wl = 3;
        // 2^(bits_log2 - 5) words of 32 bits per block
        const uint32_t bl = ctx->tune.text_filter_bits_log2;
        const uint64_t need = bl >= 5 ? h_tcount[t] << (bl - 5) : (h_tcount[t] + 1) >> (5 - bl);
        while ((1ull << wl) < need) ++wl;
        h_wl[t] = wl;
        h_off[t] = tf_total;
        tf_total += 1ull << wl;
        if (wl > tf_lds) {
          h_foff[t] = (uint64_t)h_big.size() << tf_lds;
          h_big.push_back(t);
        }
      }
      nbig = (uint32_t)h_big.size();
      tf_words = alloc<uint32_t>(ctx, tf_total);
      tf_off = alloc<uint64_t>(ctx, T);
      tf_wl = alloc<uint32_t>(ctx, T);
      span_ctr = alloc<uint64_t>(ctx, 1);
      upload(ctx, tf_off.p, h_off.data(), T);
      upload(ctx, tf_wl.p, h_wl.data(), T);
      if (nbig) {
        tf_fold = alloc<uint32_t>(ctx, (uint64_t)nbig << tf_lds);
        tf_fold_off = alloc<uint64_t>(ctx, T);
        tf_big = alloc<uint32_t>(ctx, nbig);
        upload(ctx, tf_fold_off.p, h_foff.data(), T);
        upload(ctx, tf_big.p, h_big.data(), nbig);
      }
    }

    // nkeys: keys of the phase (pairs of consecutive blocks, or unmarked blocks)
    auto run_phase = [&](int phase, uint64_t nkeys) {
      a.phase = phase;
      a.pc = ctx->profile ? pstats.p + (2 * (uint64_t)step + (phase - 1)) * kPcWords : nullptr;
      if (ctx->profile) phase_host.push_back({step, b, (uint64_t)phase, c});
      a.Lmain = phase == 1 ? 2 * b : b;
      a.xLmain = host_pow61(x, a.Lmain);
      // LDS filter: about 32 bits per key, at most 2^19 (64 KiB), two bits per
      // key while there are at least 8 bits per key.  The scan tests the
      // 32-bit pre-filter hash and queues its candidates (mode 1); from 2^14
      // keys on, where the LDS filter starts to pass a sizeable share of the
      // windows, those also test a blocked second filter in global memory of
      // about 32 bits per key (at most 2^24 bits, L2-resident; beyond 2^19
      // keys it is what rejects most windows).  Queue entries pack a position
      // below 2^40 and a text below 2^24; past that, a 2^19-bit filter on
      // 61-bit fingerprints without queues (mode 2), whose passes probe the
      // table at once.
      fbits = 12;
      while (fbits < 19 && (1ull << fbits) < 32 * nkeys) ++fbits;
      uint32_t f2words = 0;
      const bool can_queue = T <= (1u << 24) && offs[T] < (1ull << 40) &&
                             !(prm.debug_flags & BT_DBG_NO_QUEUE);
      if (can_queue) {
        scan_mode = 1;
        if (nkeys >= (1ull << 14)) {  // 64-bit words, about 32 bits per key
          f2words = 10;
          while (f2words < ctx->tune.filter2_max_log2 - 6 && (64ull << f2words) < 32 * nkeys) ++f2words;
        }
      } else {
        scan_mode = 2;
        fbits = 19;
      }
      // The byte scan: phase 1 of the upper levels, whose few keys (pairs of
      // 2b >= 32 bytes, short final pairs of more than b) are all at least 8
      // bytes long.  A filter of the keys' first eight bytes replaces the hash
      // filters.  Its queue entries pack a position below 2^40, a text below
      // 2^23 and a fit bit.  (Measured: with more keys, or in phase 2, the
      // windows that share a key's first eight bytes cost more than the hash
      // filters save.)
      const bool byte_scan = phase == 1 && b >= 16 && nkeys <= 128 && T < (1u << 23) &&
                             offs[T] < (1ull << 40) && !(prm.debug_flags & BT_DBG_NO_BYTE_SCAN);
      uint32_t bbits = 0;
      if (byte_scan) {
        // at least 2048 bits per key (chance passes below 1/2048 of windows);
        // every workgroup copies the filter into LDS
        bbits = 12;
        while (bbits < 19 && (1ull << bbits) < 2048 * nkeys) ++bbits;
        fbits = 0;
        f2words = 0;
        scan_mode = 1;
      }
      // batches: each window against its own text's filter (probe_text.hip)
      const bool text_local = tf_total && !byte_scan && scan_mode == 1;
      if (text_local) {
        fbits = 0;
        f2words = 0;
      }
      a.tf_words = text_local ? tf_words.p : nullptr;
      a.tf_off = text_local ? tf_off.p : nullptr;
      a.tf_wl = text_local ? tf_wl.p : nullptr;
      a.tf_fold = text_local ? tf_fold.p : nullptr;
      a.tf_fold_off = text_local ? tf_fold_off.p : nullptr;
      a.filt_bits = fbits;
      a.filt_two = fbits && 8 * nkeys <= (1ull << fbits);
      a.pre32 = !byte_scan && scan_mode == 1;
      a.filt2_words = f2words;
      a.bfilt = byte_scan ? filt.p : nullptr;
      a.bfilt_bits = bbits;
      a.x32L = host_pow32(x32, a.Lmain);
      a.x32Lm1 = host_pow32(x32, a.Lmain ? a.Lmain - 1 : 0);
      {
        FillList f;
        f.add(tab.p, 4 * cap, ~0u);  // empty slots: fp = best = ~0
        f.add(oddb.p, 14 * (uint64_t)T, 0);
        f.add(vcnt.p, 4, 0);
        f.add(filt.p, (1ull << (byte_scan ? bbits : fbits)) / 32, 0);
        if (f2words) f.add(filt2.p, 2ull << f2words, 0);
        if (text_local) {
          f.add(tf_words.p, tf_total, 0);
          f.add(span_ctr.p, 2, 0);
        }
        HIPCHK(ctx, launch_fill_many(f, s));
      }
      HIPCHK(ctx, launch_keys(a, s));
      // no keys: the slots say so (kNoKey), and there is nothing to scan for
      if (nkeys == 0) return;
      if (text_local) HIPCHK(ctx, launch_fold_filters(a, tf_big.p, nbig, s));
      PhaseArgs as = a;  // the scan walks segments in place of runs
      uint64_t* swoff = woff.p;
      uint64_t* wst = wstats.p + 2 * step + (phase - 1);
      if (phase == 1) {
        HIPCHK(ctx, launch_segments(a, sg, woff.p, s));
        scan(woff.p, E_ent);
        as.lv.R = E_ent;
        as.lv.rs = seg_ws.p;
        as.lv.re = seg_re.p;
        as.lv.rtext = seg_text.p;
        if (E_ent && E_ent <= c) {
          // entries whose starts continue the previous entry's join its
          // segment (phase 2's segment arrays are free until then)
          HIPCHK(ctx, launch_seg_heads(sg, woff.p, bhd.p, s));
          scan(bhd.p, E_ent);
          HIPCHK(ctx, launch_seg_merge(sg, woff.p, bhd.p, bws.p, bre.p, btext.p, bwoff.p, s));
          swoff = bwoff.p;
          as.lv.rs = bws.p;
          as.lv.re = bre.p;
          as.lv.rtext = btext.p;
        }
      } else {
        HIPCHK(ctx, launch_block_seg_counts(a, facts.p, bwc.p, bhd.p, s));
        scan(bwc.p, c);
        scan(bhd.p, c);
        HIPCHK(ctx, launch_block_segments(a, bwc.p, bhd.p, bws.p, bre.p, btext.p, bwoff.p, s));
        swoff = bwoff.p;
        as.lv.R = c;
        as.lv.rs = bws.p;
        as.lv.re = bre.p;
        as.lv.rtext = btext.p;
      }
      if (ctx->profile)  // window count of the launch, for the kernel statistics
        HIPCHK(ctx, hipMemcpyAsync(wst, swoff + as.lv.R, 8, hipMemcpyDeviceToDevice, s));
      // algorithmic bytes per window: the two prefix values it reads (8-byte
      // 61-bit prefixes, or 4-byte 32-bit hashes when pre-filtering)
      if (prm.debug_flags & BT_DBG_SORT_PHASES) {
        // Section 5.1: sort (fingerprint, position) of every window and key
        std::vector<uint64_t> wv;
        read_words(ctx, {{swoff + as.lv.R, 1}}, wv);
        const uint64_t W = wv[0], n2 = W + c;
        if (n2 >= (1ull << 31)) {
          ctx->err = "sort-based phase: 2^31 windows or more";
          throw Fail{BT_E_INVAL};
        }
        const uint64_t none = (a.fpmask == ~0ull) ? (1ull << 61) : a.fpmask + 1;
        int end_bit = 1;
        while (end_bit < 64 && (1ull << end_bit) <= none) ++end_bit;
        Buf<uint64_t> f1 = alloc<uint64_t>(ctx, n2), p1 = alloc<uint64_t>(ctx, n2),
                      f2 = alloc<uint64_t>(ctx, n2), p2 = alloc<uint64_t>(ctx, n2),
                      gx = alloc<uint64_t>(ctx, n2 + 1), gf = alloc<uint64_t>(ctx, n2);
        size_t tb = 0;
        HIPCHK(ctx, sort_pairs_u64(nullptr, tb, f1.p, f2.p, p1.p, p2.p, n2, end_bit, s));
        Buf<uint8_t> tmp = alloc<uint8_t>(ctx, tb);
        timed(ctx, "sort_phase", 0, 0, nullptr, 0, [&] {
          hipError_t e = launch_sort_emit(as, swoff, W, none, f1.p, p1.p, s);
          if (e == hipSuccess) e = sort_pairs_u64(tmp.p, tb, f1.p, f2.p, p1.p, p2.p, n2, end_bit, s);
          if (e == hipSuccess) e = launch_sort_heads(f2.p, n2, gx.p, s);
          if (e != hipSuccess) return e;
          scan(gx.p, n2);  // group numbers
          return launch_sort_groups(a, f2.p, p2.p, gx.p, n2, gf.p, s);
        });
      } else if (byte_scan) {
        // algorithmic bytes per window: the one text byte each window start adds
        timed(ctx, "byte_scan", 0, 0, wst, 1.0, [&] {
          return launch_byte_scan(as, swoff, has_odd, has_salt, c * b, s);
        }, a.Lmain);
      } else {
        // A wave's tile is kProbeTile consecutive windows, whose two reads cover
        // prefix values [i0, i0 + tile) and [i0 + L, i0 + L + tile): the bytes
        // the tile must fetch are those of the union, so the partner read is
        // counted only for the part beyond the tile.
        const double per_value = a.pre32 ? 4.0 : 8.0;
        const double partner = (double)std::min<uint64_t>(a.Lmain, kProbeTile) / (double)kProbeTile;
        // spans: at least four per resident workgroup (256) for the level's
        // window bound, 16 to 256 chunks, a multiple of the 16 waves
        uint64_t span_chunks = (c * b) / kProbeTile / (4 * 256);
        span_chunks = std::min<uint64_t>(256, std::max<uint64_t>(16, span_chunks & ~15ull));
        if (ctx->tune.span_chunks) span_chunks = ctx->tune.span_chunks;
        Buf<uint64_t> span_info;
        if (text_local) {
          span_info = alloc<uint64_t>(ctx, 3 * probe_text_spans(c * b, span_chunks));
          HIPCHK(ctx, launch_span_info(as, swoff, c * b, span_chunks, span_info.p, s));
        }
        timed(ctx, "probe_scan", 0, 0, wst, per_value * (1.0 + partner), [&] {
          // phase 2's segments (runs of blocks whose pairs do not occur
          // earlier) are short against a tile at the lowest levels
          return text_local ? launch_probe_text(as, swoff, has_odd, c * b, span_chunks, span_ctr.p,
                                                span_info.p, phase == 2 && b <= 64, s)
                            : launch_probe_scan(as, swoff, has_odd, has_salt, c * b, scan_mode, s);
        }, a.Lmain);
      }
      HIPCHK(ctx, launch_resolve(a, vb, s));
      timed(ctx, "verify", 0, 0, nullptr, 0, [&] { return launch_verify(a, vb, a.Lmain, s); });
      HIPCHK(ctx, launch_finish(a, vb, s));
      HIPCHK(ctx, launch_retry(a, vb, s));
      if (a.pc) HIPCHK(ctx, launch_phase_record(a.pc, wst, vb, s));
    };

    // ---- phase 1: pairs (a3, a4) and marks (a5)
    a.all_blocks = 0;
    run_phase(1, c - R);
    Buf<uint64_t> uoff = alloc<uint64_t>(ctx, c + 1), nrun = alloc<uint64_t>(ctx, c + 1);
    HIPCHK(ctx, launch_mark_facts(a, marked.p, facts.p, uoff.p, nrun.p, s));

    // ---- phase 2: unmarked blocks (a6) and pointers (a7)
    scan(uoff.p, c);
    std::vector<uint64_t> uu;
    read_words(ctx, {{uoff.p + c, 1}, {roff.p + c, 1}}, uu);
    check_runs(uu[1], R);
    // When most blocks are unmarked the phase-2 scan costs the same with a key
    // for every block; the leftmost occurrences of the marked blocks then tell
    // the next level which windows are copies.  Not worth it before the last
    // scanned level.
    // Pruning needs every block's leftmost occurrence, so it asks for all.
    a.all_blocks = (prune || (4 * uu[0] >= c && step + 2 < H)) ? 1 : 0;
    run_phase(2, a.all_blocks ? c : uu[0]);
    if (a.all_blocks) HIPCHK(ctx, launch_block_facts(a, facts.p, s));
    // pointers of the unmarked blocks, compacted by unmarked rank: tree storage
    // (with pruning, written once the marks are final)
    Buf<uint64_t> spb, spo;
    if (!prune) {
      spb = alloc<uint64_t>(ctx, uu[0]);
      spo = alloc<uint64_t>(ctx, uu[0]);
      HIPCHK(ctx, launch_pointers(a, marked.p, uoff.p, d_tfirst.p, spb.p, spo.p,
                                  reinterpret_cast<uint32_t*>(d_err.p), s));
    }

    // ---- split (a8): per-text counts of the next level
    const uint64_t bn = b / prm.tau;
    Buf<uint64_t> cs = alloc<uint64_t>(ctx, c + 1);
    HIPCHK(ctx, launch_child_counts(lv, tx, marked.p, bn, cs.p, s));
    scan(cs.p, c);
    std::vector<uint32_t> ids;
    std::vector<uint64_t> ent;
    entering(step + 1, ids, ent, bn);
    Buf<uint64_t> d_ent = alloc<uint64_t>(ctx, T);
    upload(ctx, d_ent.p, ent.data(), T);
    Buf<uint64_t> ntcount = alloc<uint64_t>(ctx, T + 1), ntfirst = alloc<uint64_t>(ctx, T + 1);
    Buf<uint64_t> tu = alloc<uint64_t>(ctx, T);
    if (T <= kTextStepMax) {  // counts, their prefix and the unmarked deltas in one launch
      HIPCHK(ctx, launch_text_step(T, cs.p, d_tfirst.p, d_tcount.p, d_ent.p, uoff.p, ntcount.p,
                                   ntfirst.p, tu.p, s));
    } else {
      HIPCHK(ctx, launch_text_counts(T, cs.p, d_tfirst.p, d_tcount.p, d_ent.p, ntcount.p, s));
      HIPCHK(ctx, hipMemcpyAsync(ntfirst.p, ntcount.p, T * 8, hipMemcpyDeviceToDevice, s));
      scan(ntfirst.p, T);
      HIPCHK(ctx, launch_text_deltas(uoff.p, d_tfirst.p, d_tcount.p, T, tu.p, s));
    }
    scan(nrun.p, c);
    std::vector<uint64_t> got;
    read_words(ctx, {{ntcount.p, T}, {tu.p, T}, {uoff.p + c, 1}, {nrun.p + c, 1}}, got);
    std::vector<uint64_t> h_ntcount(got.begin(), got.begin() + T);
    std::vector<uint64_t> h_tu(got.begin() + T, got.begin() + 2 * T);
    const uint64_t u = got[2 * T];
    R_pred = got[2 * T + 1];  // runs of the next level: groups of marked blocks ...
    for (uint32_t t : ids) R_pred += ent[t] ? 1 : 0;  // ... and non-empty entering texts

    // ---- outputs of this level: marks (word range per text) and pointers
    if (!prune)
      store_level(step, b, c, st.p, text.p, marked.p, uoff.p, spb, spo, u, h_tcount, h_tfirst,
                  h_tu, d_tfirst.p, d_tcount.p);

    // ---- next level's blocks
    uint64_t cn = 0;
    for (uint32_t t = 0; t < T; ++t) cn += h_ntcount[t];
    Buf<uint64_t> nst = alloc<uint64_t>(ctx, cn);
    Buf<uint32_t> ntext = alloc<uint32_t>(ctx, cn);
    HIPCHK(ctx, launch_write_children(lv, tx, marked.p, bn, prm.tau, cs.p, d_tfirst.p, ntfirst.p,
                                      nst.p, ntext.p, s));
    Buf<uint32_t> d_ids = alloc<uint32_t>(ctx, ids.size());
    upload(ctx, d_ids.p, ids.data(), ids.size());
    HIPCHK(ctx, launch_write_entering(d_ids.p, (uint32_t)ids.size(), tx, bn, ntfirst.p, nst.p,
                                      ntext.p, s));
    {
      const uint64_t nmarked = c - u;
      const uint64_t En = nmarked + ids.size();
      Buf<uint64_t> na = alloc<uint64_t>(ctx, En), ne = alloc<uint64_t>(ctx, En),
                    nchild = alloc<uint64_t>(ctx, En);
      Buf<uint8_t> nf = alloc<uint8_t>(ctx, En);
      HIPCHK(ctx, launch_entries_next(lv, tx, marked.p, facts.p, uoff.p, cs.p, d_tfirst.p,
                                      ntfirst.p, nmarked, d_ids.p, (uint32_t)ids.size(), na.p,
                                      ne.p, nf.p, nchild.p, s));
      E_ent = En;
      ent_a = std::move(na);
      ent_e = std::move(ne);
      ent_f = std::move(nf);
      ent_child = std::move(nchild);
      have_entries = true;
    }
    if (prune) {
      PruneLevel& K = pl[step];
      K.b = b;
      K.c = c;
      K.st = std::move(st);
      K.text = std::move(text);
      K.run = std::move(run);
      K.marked = std::move(marked);
      K.lm = std::move(klm);
      K.cs = std::move(cs);
      K.tfirst = std::move(d_tfirst);
      K.tcount = std::move(d_tcount);
      K.h_tcount = h_tcount;
      K.h_tfirst = h_tfirst;
    }
    std::swap(d_tcount, ntcount);
    std::swap(d_tfirst, ntfirst);
    h_tcount = h_ntcount;
    for (uint32_t t = 0; t < T; ++t) h_tfirst[t + 1] = h_tfirst[t] + h_tcount[t];
    st = std::move(nst);
    text = std::move(ntext);
    c = cn;
  }

  // ---- optional pruning (Section 4.1), deepest internal level first.  A
  // level's decisions need its children's final marks; a level's block set is
  // final once the level above has been decided, and is stored then.
  if (prune) {
    uint32_t* err = reinterpret_cast<uint32_t*>(d_err.p);
    Buf<uint64_t> open = alloc<uint64_t>(ctx, 1);
    // drop the blocks flagged in gone (null: none) from level `step` and store it
    auto compact_store = [&](uint32_t step, const uint8_t* gone) {
      PruneLevel& K = pl[step];
      const bool leaf = step + 1 == H;
      const uint64_t c0 = K.c;
      Buf<uint8_t> none;
      if (!gone) {
        none = alloc<uint8_t>(ctx, c0);
        HIPCHK(ctx, launch_fill_u8(none.p, 0, c0, s));
        gone = none.p;
      }
      Buf<uint64_t> keep = alloc<uint64_t>(ctx, c0 + 1), unmk = alloc<uint64_t>(ctx, c0 + 1);
      HIPCHK(ctx, launch_keep_flags(gone, leaf ? nullptr : K.marked.p, c0, keep.p, unmk.p, s));
      scan(keep.p, c0);
      scan(unmk.p, c0);
      Buf<uint64_t> ntf = alloc<uint64_t>(ctx, T + 1), ntc = alloc<uint64_t>(ctx, T + 1),
                    ntu = alloc<uint64_t>(ctx, T + 1);
      HIPCHK(ctx, launch_gather_firsts(keep.p, K.tfirst.p, T, ntf.p, s));
      HIPCHK(ctx, launch_text_deltas(keep.p, K.tfirst.p, K.tcount.p, T, ntc.p, s));
      HIPCHK(ctx, launch_text_deltas(unmk.p, K.tfirst.p, K.tcount.p, T, ntu.p, s));
      Buf<uint64_t> nst = alloc<uint64_t>(ctx, c0), nlm = alloc<uint64_t>(ctx, c0),
                    nuoff = alloc<uint64_t>(ctx, c0 + 1);
      Buf<uint32_t> ntext = alloc<uint32_t>(ctx, c0);
      Buf<uint8_t> nmarked = alloc<uint8_t>(ctx, c0);
      CompactDev cd{c0,      keep.p,  unmk.p,   K.st.p,   K.text.p, leaf ? nullptr : K.marked.p,
                    leaf ? nullptr : K.lm.p,    nst.p,    ntext.p,  nmarked.p,
                    nlm.p,   nuoff.p};
      HIPCHK(ctx, launch_compact(cd, s));
      std::vector<uint64_t> got;
      read_words(ctx, {{ntc.p, T}, {ntu.p, T}, {keep.p + c0, 1}, {unmk.p + c0, 1}}, got);
      std::vector<uint64_t> tc(got.begin(), got.begin() + T), tu(got.begin() + T, got.begin() + 2 * T);
      std::vector<uint64_t> tf(T + 1, 0);
      for (uint32_t t = 0; t < T; ++t) tf[t + 1] = tf[t] + tc[t];
      const uint64_t c = got[2 * T], u = got[2 * T + 1];
      if (leaf) {
        store_leaf_level(step, K.b, c, nst.p, ntext.p, tc, tf, ntf.p, ntc.p, nullptr, 0);
      } else {
        // runs of the stored level: a pointer that spills names two consecutive blocks
        Buf<uint64_t> roff = alloc<uint64_t>(ctx, c + 1), rs = alloc<uint64_t>(ctx, c),
                      re = alloc<uint64_t>(ctx, c);
        Buf<uint32_t> run = alloc<uint32_t>(ctx, c), rtext = alloc<uint32_t>(ctx, c);
        HIPCHK(ctx, launch_run_flags(nst.p, ntext.p, c, K.b, roff.p, s));
        scan(roff.p, c);
        HIPCHK(ctx, launch_run_table(nst.p, ntext.p, c, K.b, tx, roff.p, run.p, rs.p, re.p,
                                     rtext.p, s));
        PhaseArgs pa{};
        pa.tx = tx;
        pa.lv = LevelDev{c, K.b, nst.p, ntext.p, run.p, 0, rs.p, re.p, rtext.p};
        pa.k.lm = nlm.p;
        Buf<uint64_t> spb = alloc<uint64_t>(ctx, u), spo = alloc<uint64_t>(ctx, u);
        if (c) HIPCHK(ctx, launch_pointers(pa, nmarked.p, nuoff.p, ntf.p, spb.p, spo.p, err, s));
        store_level(step, K.b, c, nst.p, ntext.p, nmarked.p, nuoff.p, spb, spo, u, tc, tf, tu,
                    ntf.p, ntc.p);
      }
      K = PruneLevel{};
    };
    for (int step = (int)H - 2; step >= 0; --step) {
      PruneLevel& L = pl[step];
      PruneLevel& C = pl[step + 1];
      const bool child_leaf = step + 2 == (int)H;
      const uint64_t c = L.c;
      Buf<uint8_t> tgt = alloc<uint8_t>(ctx, c), state = alloc<uint8_t>(ctx, c);
      Buf<uint64_t> tinfo = alloc<uint64_t>(ctx, c);
      Buf<uint32_t> pending = alloc<uint32_t>(ctx, c);
      Buf<uint8_t> cgone = alloc<uint8_t>(ctx, C.c);
      HIPCHK(ctx, launch_fill_u8(tgt.p, 0, c, s));
      HIPCHK(ctx, launch_fill_u8(cgone.p, 0, C.c, s));
      PruneDev d{};
      d.lv = LevelDev{c, L.b, L.st.p, L.text.p, L.run.p, 0, nullptr, nullptr, nullptr};
      d.tx = tx;
      d.lm = L.lm.p;
      d.marked = L.marked.p;
      d.tgt = tgt.p;
      d.state = state.p;
      d.tinfo = tinfo.p;
      d.pending = pending.p;
      d.counters = open.p;
      d.cmarked = child_leaf ? nullptr : C.marked.p;
      d.cgone = cgone.p;
      d.cs = L.cs.p;
      d.tfirst = L.tfirst.p;
      d.ctfirst = C.tfirst.p;
      d.err = err;
      HIPCHK(ctx, launch_prune_decide_begin(d, s));
      // every round settles at least one candidate
      for (uint64_t round = 0;; ++round) {
        HIPCHK(ctx, launch_prune_round(d, s));
        std::vector<uint64_t> left;
        read_words(ctx, {{open.p, 1}}, left);
        if (!left[0]) break;
        if (round > c) {
          ctx->err = "internal: pruning rounds do not settle";
          throw Fail{BT_E_INTERNAL};
        }
      }
      HIPCHK(ctx, launch_prune_apply(d, s));
      compact_store((uint32_t)step + 1, cgone.p);
    }
    compact_store(0, nullptr);
  }

  std::vector<uint64_t> fin;
  const uint64_t npw = ctx->profile ? 2 * (uint64_t)H * kPcWords : 0;
  read_words(ctx, {{d_err.p, 1}, {wstats.p, ctx->profile ? 2 * (uint64_t)H + 2 : 0},
                   {pstats.p, npw}}, fin);
  if (ctx->profile) {
    collect_events(ctx, wstats.p, fin.data() + 1, 2 * (uint64_t)H + 2);
    const uint64_t* pw = fin.data() + 1 + 2 * (uint64_t)H + 2;
    for (const auto& ph : phase_host) {
      if (ctx->phases.size() >= kLaunchLogMax) break;
      const uint64_t* r = pw + (2 * ph[0] + (ph[2] - 1)) * kPcWords;
      ctx->phases.push_back({{ph[0], ph[1], ph[2], ph[3], r[kPcKeys], r[kPcWindows], r[kPcCand],
                              r[kPcVerified], r[kPcCollisions]}});
    }
  }
  if (fin[0]) {
    ctx->err = "device check failed: a pointer does not target a marked block or pair";
    return BT_E_INTERNAL;
  }

  // ---- trees
  // a tree's counts on one level: absolute for the whole step, absolute rows of
  // its first level, or relative
  auto rank_level = [&](TreeLevel& tl, const LevelBufs& L, uint32_t t, uint32_t l, uint64_t first) {
    if (L.acnt) tl.acnt = L.acnt + first * S;
    else if (l == 0) tl.acnt = L.aroot + L.root_row[t] * S;
    else tl.qc = L.qc + first * S * L.qw;
    tl.qw = L.qw;
    tl.st = L.st + first;
  };
  for (uint32_t t = 0; t < T; ++t) {
    bt_tree* tr = new bt_tree;
    tr->store = store;
    tr->dev = ctx->dev;
    tr->n = h_n[t];
    tr->b1 = plan[t].b1;
    tr->tau = prm.tau;
    tr->leaf = prm.leaf_len;
    tr->h = plan[t].h;
    const uint32_t e = H - plan[t].h;
    for (uint32_t l = 0; l + 1 < plan[t].h; ++l) {
      const TextLevelRec& r = rec[t][l];
      const LevelBufs& L = lbufs[e + l];
      TreeLevel tl;
      tl.b = r.b;
      tl.c = r.c;
      tl.u = r.u;
      tl.words = L.words + r.word_off;
      tl.wrank = L.wrank + r.word_off;
      tl.pb = L.pb + r.ptr_off;
      tl.po = L.po + r.ptr_off;
      if (rank_on) {
        rank_level(tl, L, t, l, r.first);
        tl.pc = L.pc + r.ptr_off * S * L.pw;
        tl.pw = L.pw;
        // marked blocks before this text's: its blocks before, less its unmarked ones
        tl.msel = L.msel + (r.first - r.ptr_off);
      }
      tr->lv.push_back(tl);
    }
    TreeLevel leafl;
    leafl.b = rec[t].back().b;
    leafl.c = rec[t].back().c;
    if (rank_on) rank_level(leafl, lbufs.back(), t, plan[t].h - 1, rec[t].back().first);
    tr->lv.push_back(leafl);
    tr->has_rank = with_rank;
    tr->sym = d_sym;
    tr->S = S;
    tr->total = d_Rtot ? d_Rtot + (uint64_t)t * S : nullptr;
    tr->tstart = h_n[t] ? offs[t] : offs[t];
    tr->leaves = leaves + leaf_off[t];
    tr->leaf_bytes = leaf_bytes[t];
    outs[t] = tr;
  }
  // query level tables of every tree, in one upload
  {
    std::vector<QLevel> ql;
    std::vector<uint64_t> at(T);
    for (uint32_t t = 0; t < T; ++t) {
      at[t] = ql.size();
      for (const TreeLevel& L : outs[t]->lv)
        ql.push_back(QLevel{L.b, L.c, L.words, L.wrank, L.pb, L.po, L.acnt, L.qc, L.pc, L.msel,
                            L.st, L.qw, L.pw});
    }
    Buf<QLevel> d = alloc<QLevel>(ctx, ql.size());
    const uint64_t words = (ql.size() * sizeof(QLevel) + 7) / 8;
    uint64_t* stg = small_host(ctx, words);
    std::memcpy(stg, ql.data(), ql.size() * sizeof(QLevel));
    HIPCHK(ctx, hipMemcpyAsync(d.p, stg, ql.size() * sizeof(QLevel), hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    QLevel* base = store->add(std::move(d), ql.size());
    for (uint32_t t = 0; t < T; ++t) {
      outs[t]->d_levels = base + at[t];
      outs[t]->dev_bytes = store->bytes / T;
      outs[t]->rank_bytes = rank_bytes / T;
    }
  }
  return BT_OK;
}

int guarded(bt_ctx* ctx, const std::function<int()>& f) {
  try {
    return f();
  } catch (const Fail& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return BT_E_NOMEM;
  }
}

QTree qtree_of(const bt_tree* t) {
  QTree q{};
  q.lv = t->d_levels;
  q.h = t->h;
  q.tau = t->tau;
  q.n = t->n;
  q.leaves = t->leaves;
  q.leaf_len = t->leaf;
  q.sym = t->sym;
  q.S = t->S;
  q.total = t->total;
  q.tstart = t->tstart;
  return q;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

int bt_ctx_create(int device, void* hip_stream, bt_ctx** out) {
  return bt_ctx_create_ex(device, hip_stream, nullptr, out);
}

int bt_ctx_create_ex(int device, void* hip_stream, const bt_allocator* allocator, bt_ctx** out) {
  if (!out) return BT_E_INVAL;
  if (allocator && (!allocator->alloc || !allocator->free)) return BT_E_INVAL;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return BT_E_INVAL;
  if (hipSetDevice(device) != hipSuccess) return BT_E_DEVICE;
  scratch_setup(device);
  bt_ctx* c = new (std::nothrow) bt_ctx;
  if (!c) return BT_E_NOMEM;
  c->dev = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->pool = std::make_shared<Pool>(device, allocator, c->stream);
  if (hipHostMalloc((void**)&c->h_tab, sizeof(PfTab), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return BT_E_NOMEM;
  }
  *out = c;
  return BT_OK;
}

void bt_ctx_destroy(bt_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->dev);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& p : ctx->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : ctx->ev_free) (void)hipEventDestroy(e);
  if (ctx->h_small) (void)hipHostFree(ctx->h_small);
  if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
  if (ctx->h_tab) (void)hipHostFree(ctx->h_tab);
  ctx->pool->trim();
  delete ctx;
}

const char* bt_ctx_last_error(const bt_ctx* ctx) {
  return ctx ? ctx->err.c_str() : "null context";
}

int bt_ctx_trim(bt_ctx* ctx) {
  if (!ctx) return BT_E_INVAL;
  ctx->pool->trim();
  return BT_OK;
}

int bt_ctx_profile(bt_ctx* ctx, int enable) {
  if (!ctx) return BT_E_INVAL;
  ctx->profile = enable != 0;
  return BT_OK;
}

int bt_ctx_kernel_stats(const bt_ctx* ctx, const char* name, uint64_t* launches, double* total_ms,
                        double* bytes, double* units) {
  if (!ctx || !name) return BT_E_INVAL;
  auto it = ctx->stats.find(name);
  KStat z;
  const KStat& k = it == ctx->stats.end() ? z : it->second;
  if (launches) *launches = k.launches;
  if (total_ms) *total_ms = k.ms;
  if (bytes) *bytes = k.bytes;
  if (units) *units = k.units;
  return BT_OK;
}

int bt_ctx_reset_stats(bt_ctx* ctx) {
  if (!ctx) return BT_E_INVAL;
  ctx->stats.clear();
  ctx->launches.clear();
  ctx->phases.clear();
  return BT_OK;
}

int bt_ctx_set_tuning(bt_ctx* ctx, const bt_tuning* t) {
  if (!ctx || !t) return BT_E_INVAL;
  if (t->table_load_log2 < 1 || t->table_load_log2 > 3 || t->text_filter_bits_log2 < 4 ||
      t->text_filter_bits_log2 > 7 || t->span_chunks > 1024 || (t->span_chunks & 15) ||
      t->filter2_max_log2 < 16 || t->filter2_max_log2 > 28) {
    ctx->err = "bt_ctx_set_tuning: a value outside its documented range";
    return BT_E_INVAL;
  }
  ctx->tune = *t;
  return BT_OK;
}

int bt_ctx_get_tuning(const bt_ctx* ctx, bt_tuning* t) {
  if (!ctx || !t) return BT_E_INVAL;
  *t = ctx->tune;
  return BT_OK;
}

int bt_ctx_phase_count(const bt_ctx* ctx, uint64_t* count) {
  if (!ctx || !count) return BT_E_INVAL;
  *count = ctx->phases.size();
  return BT_OK;
}

int bt_ctx_phase_record(const bt_ctx* ctx, uint64_t idx, uint64_t* rec) {
  if (!ctx || !rec || idx >= ctx->phases.size()) return BT_E_INVAL;
  std::memcpy(rec, ctx->phases[idx].v, sizeof(ctx->phases[idx].v));
  return BT_OK;
}

int bt_ctx_launch_count(const bt_ctx* ctx, uint64_t* count) {
  if (!ctx || !count) return BT_E_INVAL;
  *count = ctx->launches.size();
  return BT_OK;
}

int bt_ctx_launch_record(const bt_ctx* ctx, uint64_t idx, char* name, uint64_t name_cap,
                         uint64_t* window_len, double* units, double* ms, double* bytes) {
  if (!ctx || idx >= ctx->launches.size()) return BT_E_INVAL;
  const LaunchRec& r = ctx->launches[idx];
  if (name && name_cap) {
    const size_t k = std::min<size_t>(r.name.size(), name_cap - 1);
    std::memcpy(name, r.name.data(), k);
    name[k] = 0;
  }
  if (window_len) *window_len = r.wlen;
  if (units) *units = r.units;
  if (ms) *ms = r.ms;
  if (bytes) *bytes = r.bytes;
  return BT_OK;
}

int bt_ctx_memory(const bt_ctx* ctx, uint64_t* in_use, uint64_t* peak, uint64_t* held) {
  if (!ctx) return BT_E_INVAL;
  if (in_use) *in_use = ctx->pool->in_use();
  if (peak) *peak = ctx->pool->peak();
  if (held) *held = ctx->pool->held();
  return BT_OK;
}

int bt_ctx_reset_peak(bt_ctx* ctx) {
  if (!ctx) return BT_E_INVAL;
  ctx->pool->reset_peak();
  return BT_OK;
}

int bt_prefix_fingerprints(bt_ctx* ctx, const uint8_t* d_text, uint64_t n, uint64_t x,
                           uint64_t* d_P) {
  if (!ctx) return BT_E_INVAL;
  if (x == 0 || x >= kP61Host || !d_P || (!d_text && n)) {
    ctx->err = "bt_prefix_fingerprints: need 1 <= x < 2^61-1 and valid pointers";
    return BT_E_INVAL;
  }
  return guarded(ctx, [&] {
    HIPCHK(ctx, hipSetDevice(ctx->dev));
    Buf<PfTab> d_tab = alloc<PfTab>(ctx, 1);
    fill_tab(ctx->h_tab, x, 1u);
    HIPCHK(ctx, hipMemcpyAsync(d_tab.p, ctx->h_tab, sizeof(PfTab), hipMemcpyHostToDevice,
                               ctx->stream));
    Buf<uint64_t> d_status = alloc<uint64_t>(ctx, prefix_status_words(n));
    timed(ctx, "prefix_fp", (double)n + 8.0 * (double)(n + 1), (double)n, nullptr, 0, [&] {
      return launch_prefix(d_text, n, d_P, false, nullptr, d_tab.p, d_status.p, ctx->stream);
    });
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    collect_events(ctx);
    return BT_OK;
  });
}

int bt_prefix_scan(bt_ctx* ctx, const uint8_t* d_text, uint64_t n, uint64_t x, uint32_t x32,
                   int sampled, uint64_t* d_P, uint32_t* d_H) {
  if (!ctx) return BT_E_INVAL;
  if (x == 0 || x >= kP61Host || !d_P || !d_H || (!d_text && n) || sampled < 0 || sampled > 2) {
    ctx->err = "bt_prefix_scan: need 1 <= x < 2^61-1, sampled 0, 1 or 2 and valid pointers";
    return BT_E_INVAL;
  }
  return guarded(ctx, [&] {
    HIPCHK(ctx, hipSetDevice(ctx->dev));
    Buf<PfTab> d_tab = alloc<PfTab>(ctx, 1);
    fill_tab(ctx->h_tab, x, x32);
    HIPCHK(ctx, hipMemcpyAsync(d_tab.p, ctx->h_tab, sizeof(PfTab), hipMemcpyHostToDevice,
                               ctx->stream));
    Buf<uint64_t> d_status = alloc<uint64_t>(ctx, prefix_status_words(n));
    const double pw = sampled ? 8.0 * (double)(n / 16 + 1) : 8.0 * (double)(n + 1);
    const double hw = sampled == 2 ? 4.0 * (double)(n / 16 + 1) : 4.0 * (double)(n + 1);
    timed(ctx, "prefix_fp", (double)n + pw + hw, (double)n, nullptr, 0, [&] {
      return launch_prefix(d_text, n, d_P, sampled != 0, d_H, d_tab.p, d_status.p, ctx->stream,
                           sampled == 2);
    });
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    collect_events(ctx);
    return BT_OK;
  });
}

int bt_prefix_scan_noalloc(bt_ctx* ctx, const uint8_t* d_text, uint64_t n, uint64_t x,
                           uint32_t x32, int sampled, uint64_t* d_P, uint32_t* d_H) {
  if (!ctx) return BT_E_INVAL;
  if (x == 0 || x >= kP61Host || !d_P || !d_H || (!d_text && n) || sampled < 0 || sampled > 2) {
    ctx->err = "bt_prefix_scan_noalloc: need 1 <= x < 2^61-1, sampled 0, 1 or 2 and valid pointers";
    return BT_E_INVAL;
  }
  if (n > kNoAllocMaxText) {
    ctx->err = "bt_prefix_scan_noalloc: texts of at most 2^33 bytes (the fixed scratch size)";
    return BT_E_INVAL;
  }
  uint64_t* base = scratch_base(ctx->dev);
  if (!base) {
    ctx->err = "bt_prefix_scan_noalloc: the fixed scratch array of this device was not found";
    return BT_E_DEVICE;
  }
  PfTab* tab = reinterpret_cast<PfTab*>(base);
  uint64_t* status = base + kNoAllocTabWords;
  hipError_t e = hipSetDevice(ctx->dev);
  if (e == hipSuccess) {
    fill_tab(ctx->h_tab, x, x32);
    e = hipMemcpyAsync(tab, ctx->h_tab, sizeof(PfTab), hipMemcpyHostToDevice, ctx->stream);
  }
  if (e == hipSuccess)
    e = launch_prefix(d_text, n, d_P, sampled != 0, d_H, tab, status, ctx->stream, sampled == 2);
  // synchronous, like bt_prefix_scan: the pinned staging of the tables and the
  // scratch are free again when the call returns
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    ctx->err = std::string("bt_prefix_scan_noalloc: ") + hipGetErrorString(e);
    return BT_E_DEVICE;
  }
  return BT_OK;
}

int bt_build_ex(bt_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t sigma,
                const bt_params* params, bt_tree** out) {
  if (!ctx) return BT_E_INVAL;
  if (!params || !out) {
    ctx->err = "null params or output";
    return BT_E_INVAL;
  }
  *out = nullptr;
  std::vector<uint64_t> offs{0, n};
  return guarded(ctx, [&] { return build_many(ctx, d_text, offs, sigma, *params, out); });
}

int bt_build(bt_ctx* ctx, const uint8_t* d_text, uint64_t n, uint32_t sigma, uint32_t tau,
             uint32_t leaf_len, bt_tree** out) {
  bt_params p{};
  p.tau = tau;
  p.leaf_len = leaf_len;
  p.s_hint = 1;
  p.hash_seed = 0x0B10C7EEull;
  p.flags = BT_WITH_RANK_SELECT;
  return bt_build_ex(ctx, d_text, n, sigma, &p, out);
}

int bt_build_batch(bt_ctx* ctx, const uint8_t* d_concat, const uint64_t* h_offsets, uint32_t num,
                   uint32_t sigma, const bt_params* params, bt_tree** outs) {
  if (!ctx) return BT_E_INVAL;
  if (!params || (num && (!h_offsets || !outs))) {
    ctx->err = "null params, offsets or outputs";
    return BT_E_INVAL;
  }
  std::vector<uint64_t> offs(h_offsets, h_offsets + (num ? num + 1 : 0));
  if (num == 0) return BT_OK;
  for (uint32_t i = 0; i < num; ++i) outs[i] = nullptr;
  return guarded(ctx, [&] { return build_many(ctx, d_concat, offs, sigma, *params, outs); });
}

int bt_tree_info(const bt_tree* t, uint64_t* n, uint32_t* h, uint64_t* b1) {
  if (!t) return BT_E_INVAL;
  if (n) *n = t->n;
  if (h) *h = t->h;
  if (b1) *b1 = t->b1;
  return BT_OK;
}

int bt_level_info(const bt_tree* t, uint32_t level, uint64_t* b, uint64_t* c, uint64_t* u) {
  if (!t || level < 1 || level > t->h) return BT_E_INVAL;
  const TreeLevel& L = t->lv[level - 1];
  if (b) *b = L.b;
  if (c) *c = L.c;
  if (u) *u = L.u;
  return BT_OK;
}

int bt_level_copy(const bt_tree* t, uint32_t level, uint64_t* marked_words, uint64_t* ptr_block,
                  uint64_t* ptr_off) {
  if (!t || level < 1 || level >= t->h) return BT_E_INVAL;
  const TreeLevel& L = t->lv[level - 1];
  if (hipSetDevice(t->dev) != hipSuccess) return BT_E_DEVICE;
  const uint64_t nw = (L.c + 63) / 64;
  if (marked_words && nw && hipMemcpy(marked_words, L.words, nw * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return BT_E_DEVICE;
  if (ptr_block && L.u && hipMemcpy(ptr_block, L.pb, L.u * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return BT_E_DEVICE;
  if (ptr_off && L.u && hipMemcpy(ptr_off, L.po, L.u * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return BT_E_DEVICE;
  return BT_OK;
}

int bt_level_copy_async(const bt_tree* t, uint32_t level, uint64_t* marked_words,
                        uint64_t* ptr_block, uint64_t* ptr_off, void* stream) {
  if (!t || level < 1 || level >= t->h) return BT_E_INVAL;
  const TreeLevel& L = t->lv[level - 1];
  if (hipSetDevice(t->dev) != hipSuccess) return BT_E_DEVICE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t nw = (L.c + 63) / 64;
  hipError_t e = hipSuccess;
  if (marked_words && nw) e = hipMemcpyAsync(marked_words, L.words, nw * 8, hipMemcpyDefault, s);
  if (e == hipSuccess && ptr_block && L.u)
    e = hipMemcpyAsync(ptr_block, L.pb, L.u * 8, hipMemcpyDefault, s);
  if (e == hipSuccess && ptr_off && L.u)
    e = hipMemcpyAsync(ptr_off, L.po, L.u * 8, hipMemcpyDefault, s);
  return e == hipSuccess ? BT_OK : BT_E_DEVICE;
}

int bt_leaves_size(const bt_tree* t, uint64_t* bytes) {
  if (!t || !bytes) return BT_E_INVAL;
  *bytes = t->leaf_bytes;
  return BT_OK;
}

int bt_leaves_copy(const bt_tree* t, uint8_t* dst) {
  if (!t || (!dst && t->leaf_bytes)) return BT_E_INVAL;
  if (!t->leaf_bytes) return BT_OK;
  if (hipSetDevice(t->dev) != hipSuccess) return BT_E_DEVICE;
  return hipMemcpy(dst, t->leaves, t->leaf_bytes, hipMemcpyDeviceToHost) == hipSuccess ? BT_OK
                                                                                   : BT_E_DEVICE;
}

int bt_serialize(const bt_tree* t, uint8_t* dst, uint64_t cap, uint64_t* written) {
  if (!t || !written) return BT_E_INVAL;
  std::vector<uint8_t> out;
  auto put = [&](const void* p, size_t k) {
    const uint8_t* q = static_cast<const uint8_t*>(p);
    out.insert(out.end(), q, q + k);
  };
  const uint32_t zero = 0;
  put("BTv1", 4);
  put(&t->n, 8);
  put(&t->tau, 4);
  put(&t->leaf, 4);
  put(&t->b1, 8);
  put(&t->h, 4);
  put(&zero, 4);
  for (uint32_t l = 1; l < t->h; ++l) {
    const TreeLevel& L = t->lv[l - 1];
    std::vector<uint64_t> w((L.c + 63) / 64), pb(L.u), po(L.u);
    int rc = bt_level_copy(t, l, w.data(), pb.data(), po.data());
    if (rc) return rc;
    put(&L.b, 8);
    put(&L.c, 8);
    put(w.data(), w.size() * 8);
    put(&L.u, 8);
    put(pb.data(), pb.size() * 8);
    put(po.data(), po.size() * 8);
  }
  const TreeLevel& Lh = t->lv[t->h - 1];
  put(&Lh.b, 8);
  put(&Lh.c, 8);
  put(&t->leaf_bytes, 8);
  std::vector<uint8_t> lb(t->leaf_bytes);
  int rc = bt_leaves_copy(t, lb.data());
  if (rc) return rc;
  put(lb.data(), lb.size());
  const uint64_t zeros = 0;
  put(&zeros, (8 - (t->leaf_bytes & 7)) & 7);
  *written = out.size();
  if (!dst) return BT_OK;
  if (cap < out.size()) return BT_E_INVAL;
  std::memcpy(dst, out.data(), out.size());
  return BT_OK;
}

int bt_access(bt_ctx* ctx, const bt_tree* t, const uint64_t* d_pos, uint64_t m, uint8_t* d_out) {
  if (!ctx || !t || (m && (!d_pos || !d_out))) return BT_E_INVAL;
  return guarded(ctx, [&] {
    HIPCHK(ctx, hipSetDevice(ctx->dev));
    Buf<uint64_t> bad = alloc<uint64_t>(ctx, 1);
    HIPCHK(ctx, launch_fill_u64(bad.p, 0, 1, ctx->stream));
    if (t->n == 0) {
      HIPCHK(ctx, launch_fill_u8(d_out, 0, m, ctx->stream));
      HIPCHK(ctx, launch_fill_u64(bad.p, m ? 1 : 0, 1, ctx->stream));
    } else {
      HIPCHK(ctx, launch_access(qtree_of(t), d_pos, m, d_out, reinterpret_cast<uint32_t*>(bad.p),
                                ctx->stream));
    }
    std::vector<uint64_t> r;
    read_words(ctx, {{bad.p, 1}}, r);
    if (r[0]) {
      ctx->err = "bt_access: position out of range";
      return BT_E_INVAL;
    }
    return BT_OK;
  });
}

int bt_rank(bt_ctx* ctx, const bt_tree* t, const uint8_t* d_c, const uint64_t* d_pos, uint64_t m,
            uint64_t* d_out) {
  if (!ctx || !t || (m && (!d_c || !d_pos || !d_out))) return BT_E_INVAL;
  if (!t->has_rank) {
    ctx->err = "bt_rank: the tree was built without BT_WITH_RANK_SELECT";
    return BT_E_INVAL;
  }
  return guarded(ctx, [&] {
    HIPCHK(ctx, hipSetDevice(ctx->dev));
    if (t->n == 0 || t->S == 0) {
      // empty text: rank(c, 0) = 0, anything else is out of range
      HIPCHK(ctx, launch_rank_empty(d_pos, m, d_out, ctx->stream));
    } else {
        HIPCHK(ctx, launch_rank(qtree_of(t), d_c, d_pos, m, d_out, ctx->stream));
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return BT_OK;
  });
}

int bt_select(bt_ctx* ctx, const bt_tree* t, const uint8_t* d_c, const uint64_t* d_k, uint64_t m,
              uint64_t* d_out) {
  if (!ctx || !t || (m && (!d_c || !d_k || !d_out))) return BT_E_INVAL;
  if (!t->has_rank) {
    ctx->err = "bt_select: the tree was built without BT_WITH_RANK_SELECT";
    return BT_E_INVAL;
  }
  return guarded(ctx, [&] {
    HIPCHK(ctx, hipSetDevice(ctx->dev));
    if (t->n == 0 || t->S == 0) {
      HIPCHK(ctx, launch_fill_u64(d_out, ~0ull, m, ctx->stream));
    } else {
        HIPCHK(ctx, launch_select(qtree_of(t), d_c, d_k, m, d_out, ctx->stream));
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return BT_OK;
  });
}

int bt_tree_device_bytes(const bt_tree* t, uint64_t* bytes) {
  if (!t || !bytes) return BT_E_INVAL;
  *bytes = t->dev_bytes;
  return BT_OK;
}

int bt_tree_rank_bytes(const bt_tree* t, uint64_t* bytes) {
  if (!t || !bytes) return BT_E_INVAL;
  *bytes = t->rank_bytes;
  return BT_OK;
}

void bt_tree_free(bt_tree* t) { delete t; }

int bt_trees_free(bt_tree* const* trees, uint64_t n) {
  if (!trees && n) return BT_E_INVAL;
  for (uint64_t i = 0; i < n; ++i) delete trees[i];
  return BT_OK;
}

const char* bt_strerror(int status) {
  switch (status) {
    case BT_OK: return "ok";
    case BT_E_INVAL: return "invalid argument";
    case BT_E_NOMEM: return "out of memory";
    case BT_E_DEVICE: return "HIP runtime error";
    case BT_E_INTERNAL: return "internal consistency check failed";
    default: return "unknown status";
  }
}

}  // extern "C"
