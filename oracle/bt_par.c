/*
 * Block-tree oracle, second construction ("T2"): the paper's own method on
 * host threads.  It is the parity reference for texts too long for the plain
 * definition in bt_oracle.c (whose direct search costs O(n) per key), and the
 * timed CPU baseline.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the GPU library.
 * Tests require it to give the same canonical bytes as the plain definition on
 * every input the definition can finish.
 *
 * What it follows:
 *   - Section 4.1, the two phases of each level: the fingerprints of all pairs
 *     of consecutive blocks go into a hash table, the level is scanned with a
 *     window of the pair length, and the leftmost occurrence of every pair is
 *     found; then the same for the unmarked blocks, giving their pointers.
 *     Each distinct key string is verified against the text once per
 *     partition; a fingerprint match is accepted only after comparing bytes.
 *   - Section 5.2 and Section 5.4, domain decomposition: the level's windows
 *     are cut into K contiguous partitions, one per thread.  Each thread keeps,
 *     per key string, only the first (locally leftmost) verified occurrence in
 *     its partition; these survivors are routed to the partition responsible
 *     for the key, chosen by its fingerprint modulo K, which keeps the global
 *     minimum.
 *   - Section 2, Karp-Rabin fingerprints phi(i, L) = sum_k T[i+k] r^(L-1-k)
 *     mod q, here with the prime q = 2^64 - 2^32 + 1 and a base r chosen by the
 *     caller; windows advance by the conventional one-step relation restated
 *     in Section 5.3.  The GPU library uses another modulus and base.  Nothing
 *     here depends on the choice: every accepted occurrence is confirmed by
 *     comparing bytes.
 *   - Windows are those lying inside a run of consecutive blocks of the level
 *     ("the leftmost occurrence on this level", Section 4).  The plain oracle
 *     searches all of T; the tests that equate the two constructions check that
 *     reading.
 * The split into tau children per marked block, the isolated-block rule and
 * the leaf level are as in bt_oracle.c (exact splits only: b1 = leaf * tau^k).
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include "ora_tree.h"

/* ---- arithmetic mod q = 2^64 - 2^32 + 1 ---- */

#define GQ 0xFFFFFFFF00000001ULL

/* x mod q for x < 2^128.  With x = lo + 2^64 (2^32 hh + hl), 2^64 = 2^32 - 1
 * and 2^96 = -1 (mod q), so x = lo - hh + hl (2^32 - 1) (mod q):
 *   t = lo - hh, adding q back on a borrow (as 64-bit words: subtract 2^32 - 1,
 *     which cannot borrow again since the wrapped value is >= 2^64 - 2^32 + 1);
 *   u = hl (2^32 - 1) = (hl << 32) - hl < 2^64;
 *   t + u, adding 2^64 mod q = 2^32 - 1 back on a carry (the wrapped sum is
 *     below 2^64 - 2^33 + 1, so this cannot carry again);
 *   one conditional subtraction of q. */
static inline uint64_t g_red(unsigned __int128 x) {
  const uint64_t lo = (uint64_t)x, hi = (uint64_t)(x >> 64);
  const uint64_t hh = hi >> 32, hl = hi & 0xFFFFFFFFu;
  uint64_t t = lo - hh;
  if (lo < hh) t -= 0xFFFFFFFFu;
  const uint64_t u = (hl << 32) - hl;
  uint64_t v = t + u;
  if (v < t) v += 0xFFFFFFFFu;
  return v >= GQ ? v - GQ : v;
}
static inline uint64_t g_mul(uint64_t a, uint64_t b) {
  return g_red((unsigned __int128)a * b);
}
static inline uint64_t g_add(uint64_t a, uint64_t b) {
  /* a, b < q: a + b < 2q; on a 64-bit carry the true sum minus q is the
   * wrapped sum plus 2^32 - 1 */
  uint64_t s = a + b;
  if (s < a) return s + 0xFFFFFFFFu;
  return s >= GQ ? s - GQ : s;
}
static inline uint64_t g_sub(uint64_t a, uint64_t b) { return a >= b ? a - b : a + (GQ - b); }

static uint64_t g_pow(uint64_t r, uint64_t e) {
  uint64_t acc = 1;
  while (e) {
    if (e & 1) acc = g_mul(acc, r);
    r = g_mul(r, r);
    e >>= 1;
  }
  return acc;
}

/* phi of T[i..i+L) by Horner's rule. */
static uint64_t phi(const uint8_t *T, uint64_t i, uint64_t L, uint64_t r) {
  uint64_t h = 0;
  for (uint64_t k = 0; k < L; ++k) h = g_add(g_mul(h, r), T[i + k]);
  return h;
}

uint64_t ora_par_window_fp(const uint8_t *T, uint64_t i, uint64_t L, uint64_t r) {
  return phi(T, i, L, r % GQ);
}

/* ---- threads: run fn(arg, t, K) for t = 0..K-1 and wait ---- */

typedef void (*par_fn)(void *arg, int t, int K);
typedef struct { par_fn fn; void *arg; int t, K; } par_job;

static void *par_trampoline(void *p) {
  par_job *j = p;
  j->fn(j->arg, j->t, j->K);
  return NULL;
}

static void par_for(int K, par_fn fn, void *arg) {
  pthread_t th[256];
  par_job jb[256];
  int started = 0;
  for (int t = 1; t < K; ++t) {
    jb[t] = (par_job){fn, arg, t, K};
    if (pthread_create(&th[t], NULL, par_trampoline, &jb[t]) != 0) break;
    started = t;
  }
  /* threads that could not be started run inline, in order */
  for (int t = started + 1; t < K; ++t) fn(arg, t, K);
  fn(arg, 0, K);
  for (int t = 1; t <= started; ++t) pthread_join(th[t], NULL);
}

/* ---- one search: leftmost occurrences of equal-length keys on a level ---- */

typedef struct { uint64_t pos; uint32_t sid; } hit;
typedef struct { hit *v; uint64_t n, cap; int oom; } hitlist;

static void hl_push(hitlist *l, uint64_t pos, uint32_t sid) {
  if (l->n == l->cap) {
    uint64_t nc = l->cap ? 2 * l->cap : 256;
    hit *nv = realloc(l->v, nc * sizeof(hit));
    if (!nv) { l->oom = 1; return; }
    l->v = nv; l->cap = nc;
  }
  l->v[l->n].pos = pos; l->v[l->n].sid = sid; ++l->n;
}

typedef struct {
  const uint8_t *T;
  uint64_t L, r;              /* window length, base */
  uint64_t out[256];          /* c r^(L-1) mod q: the term of a byte leaving the window */
  uint64_t mask;              /* fingerprint mask (all ones, or a weak mask) */
  /* keys: T[kst[k] .. kst[k]+L) */
  uint64_t nk;
  const uint64_t *kst;
  const uint64_t *kfp;        /* masked key fingerprints */
  uint32_t *ksid;             /* key -> string id */
  /* distinct key strings */
  uint64_t ns;
  uint64_t *srep, *sfp;       /* a start holding the string; its fingerprint */
  /* hash table of strings by fingerprint, and a bit filter in front of it */
  uint64_t tmask;
  uint64_t *tfp;
  uint32_t *tsid;             /* UINT32_MAX = empty */
  uint64_t *filt;
  unsigned fshift;
  /* windows: every start i with [i, i+L) inside a run [rs, re) */
  uint64_t R;
  const uint64_t *rs, *re;
  uint64_t *wpre;             /* wpre[k] = windows in runs before run k */
  /* per thread: strings already found in its partition, and the survivors
   * routed by owner (fingerprint mod K) */
  uint8_t **found;
  hitlist *route;             /* route[t * K + owner] */
  uint64_t *best;             /* per string: global leftmost */
} search_t;

static inline uint64_t mix(uint64_t fp) { return fp * 0x9E3779B97F4A7C15ULL; }

static void scan_partition(void *arg, int t, int K) {
  search_t *s = arg;
  const uint64_t W = s->wpre[s->R];
  uint64_t w = W * (uint64_t)t / K, wend = W * (uint64_t)(t + 1) / K;
  if (w >= wend) return;
  uint8_t *found = s->found[t];
  hitlist *route = s->route + (uint64_t)t * K;
  /* the run holding window w: the last k with wpre[k] <= w */
  uint64_t lo = 0, hi = s->R;
  while (hi - lo > 1) {
    uint64_t mid = (lo + hi) / 2;
    if (s->wpre[mid] <= w) lo = mid; else hi = mid;
  }
  uint64_t k = lo;
  while (w < wend) {
    while (s->wpre[k + 1] <= w) ++k;          /* skip runs with no windows */
    uint64_t i = s->rs[k] + (w - s->wpre[k]);
    uint64_t last = s->rs[k] + (s->wpre[k + 1] - s->wpre[k]) - 1;  /* last start */
    if (last > i + (wend - w) - 1) last = i + (wend - w) - 1;
    uint64_t h = phi(s->T, i, s->L, s->r);
    for (;;) {
      uint64_t fp = h & s->mask;
      uint64_t m = mix(fp) >> s->fshift;
      if (s->filt[m >> 6] >> (m & 63) & 1) {
        /* every string with this fingerprint (distinct strings may share one) */
        for (uint64_t slot = mix(fp) & s->tmask; s->tsid[slot] != UINT32_MAX;
             slot = (slot + 1) & s->tmask) {
          const uint32_t sid = s->tsid[slot];
          if (s->tfp[slot] != fp || found[sid]) continue;
          if (memcmp(s->T + i, s->T + s->srep[sid], s->L) == 0) {
            found[sid] = 1;
            hl_push(&route[s->sfp[sid] % (uint64_t)K], i, sid);
          }
        }
      }
      ++w;
      if (i == last) break;
      /* phi(i+1, L) = (phi(i, L) - T[i] r^(L-1)) r + T[i+L] */
      h = g_add(g_mul(g_sub(h, s->out[s->T[i]]), s->r), s->T[i + s->L]);
      ++i;
    }
  }
}

static void merge_owner(void *arg, int t, int K) {
  search_t *s = arg;
  for (int src = 0; src < K; ++src) {
    hitlist *l = &s->route[(uint64_t)src * K + t];
    for (uint64_t q = 0; q < l->n; ++q)
      if (l->v[q].pos < s->best[l->v[q].sid]) s->best[l->v[q].sid] = l->v[q].pos;
  }
}

/* For the nk keys T[kst[k] .. kst[k]+L) with masked fingerprints kfp[k],
 * every key lying inside one of the R runs [rs, re), write the leftmost start
 * of an equal window inside a run to out[k].  Returns ORA_OK, ORA_E_NOMEM, or
 * ORA_E_LEMMA when a key is not found (it cannot happen: the key's own window
 * lies in a run). */
static int leftmost_keys(const uint8_t *T, uint64_t L, const uint64_t *kst, const uint64_t *kfp,
                         uint64_t nk, const uint64_t *rs, const uint64_t *re, uint64_t R,
                         uint64_t r, uint64_t mask, int K, uint64_t *out) {
  if (nk == 0) return ORA_OK;
  search_t s;
  memset(&s, 0, sizeof s);
  s.T = T; s.L = L; s.r = r; s.mask = mask; s.nk = nk; s.kst = kst; s.kfp = kfp;
  s.R = R; s.rs = rs; s.re = re;
  const uint64_t rpow = g_pow(r, L - 1);
  for (int c = 0; c < 256; ++c) s.out[c] = g_mul((uint64_t)c, rpow);
  int rc = ORA_OK;
  s.ksid = malloc(nk * 4);
  s.srep = malloc(nk * 8);
  s.sfp = malloc(nk * 8);
  uint64_t cap = 1;
  while (cap < 2 * nk) cap <<= 1;
  s.tmask = cap - 1;
  s.tfp = malloc(cap * 8);
  s.tsid = malloc(cap * 4);
  /* filter: at least 16 bits per key, 2^12 bits at least */
  unsigned fb = 12;
  while (((uint64_t)1 << fb) < 16 * nk) ++fb;
  s.fshift = 64 - fb;
  s.filt = calloc(((uint64_t)1 << fb) / 64, 8);
  s.wpre = malloc((R + 1) * 8);
  s.found = calloc(K, sizeof(uint8_t *));
  s.route = calloc((uint64_t)K * K, sizeof(hitlist));
  if (!s.ksid || !s.srep || !s.sfp || !s.tfp || !s.tsid || !s.filt || !s.wpre ||
      !s.found || !s.route) { rc = ORA_E_NOMEM; goto done; }
  memset(s.tsid, 0xFF, cap * 4);

  /* distinct key strings: a key joins a string with an equal fingerprint and
   * equal bytes, else starts a new one */
  for (uint64_t k = 0; k < nk; ++k) {
    const uint64_t fp = s.kfp[k];
    uint32_t id = UINT32_MAX;
    uint64_t slot = mix(fp) & s.tmask;
    while (s.tsid[slot] != UINT32_MAX) {
      if (s.tfp[slot] == fp && memcmp(T + kst[k], T + s.srep[s.tsid[slot]], L) == 0) {
        id = s.tsid[slot];
        break;
      }
      slot = (slot + 1) & s.tmask;
    }
    if (id == UINT32_MAX) {
      id = (uint32_t)s.ns++;
      s.srep[id] = kst[k];
      s.sfp[id] = fp;
      s.tfp[slot] = fp;
      s.tsid[slot] = id;
      uint64_t m = mix(fp) >> s.fshift;
      s.filt[m >> 6] |= (uint64_t)1 << (m & 63);
    }
    s.ksid[k] = id;
  }

  /* windows per run */
  s.wpre[0] = 0;
  for (uint64_t q = 0; q < R; ++q)
    s.wpre[q + 1] = s.wpre[q] + (re[q] - rs[q] >= L ? re[q] - rs[q] - L + 1 : 0);

  for (int t = 0; t < K; ++t) {
    s.found[t] = calloc(s.ns, 1);
    if (!s.found[t]) { rc = ORA_E_NOMEM; goto done; }
  }
  s.best = malloc(s.ns * 8);
  if (!s.best) { rc = ORA_E_NOMEM; goto done; }
  for (uint64_t q = 0; q < s.ns; ++q) s.best[q] = UINT64_MAX;

  par_for(K, scan_partition, &s);
  for (uint64_t q = 0; q < (uint64_t)K * K; ++q)
    if (s.route[q].oom) { rc = ORA_E_NOMEM; goto done; }
  par_for(K, merge_owner, &s);

  for (uint64_t k = 0; k < nk; ++k) {
    out[k] = s.best[s.ksid[k]];
    if (out[k] > kst[k]) rc = ORA_E_LEMMA;
  }

done:
  if (s.found)
    for (int t = 0; t < K; ++t) free(s.found[t]);
  if (s.route)
    for (uint64_t q = 0; q < (uint64_t)K * K; ++q) free(s.route[q].v);
  free(s.found); free(s.route); free(s.best);
  free(s.ksid); free(s.srep); free(s.sfp); free(s.tfp); free(s.tsid);
  free(s.filt); free(s.wpre);
  return rc;
}

/* Leftmost occurrences of keys of mixed lengths: one search per distinct
 * length (with exact splits there are at most two: full, and one that ends
 * in the text's short final block). */
static int leftmost_mixed(const uint8_t *T, const uint64_t *kst, const uint64_t *klen,
                          const uint64_t *kfp, uint64_t nk, const uint64_t *rs,
                          const uint64_t *re, uint64_t R, uint64_t r, uint64_t mask, int K,
                          uint64_t *out) {
  uint64_t *sub = malloc((nk ? nk : 1) * 8), *subfp = malloc((nk ? nk : 1) * 8);
  uint64_t *res = malloc((nk ? nk : 1) * 8);
  uint8_t *done = calloc(nk ? nk : 1, 1);
  int rc = ORA_OK;
  if (!sub || !subfp || !res || !done) { rc = ORA_E_NOMEM; goto out; }
  for (uint64_t first = 0; first < nk; ++first) {
    if (done[first]) continue;
    const uint64_t L = klen[first];
    uint64_t m = 0;
    for (uint64_t k = first; k < nk; ++k)
      if (!done[k] && klen[k] == L) { sub[m] = kst[k]; subfp[m] = kfp[k] & mask; ++m; }
    int e = leftmost_keys(T, L, sub, subfp, m, rs, re, R, r, mask, K, res);
    if (e == ORA_E_NOMEM) { rc = e; goto out; }
    if (e != ORA_OK) rc = e;
    m = 0;
    for (uint64_t k = first; k < nk; ++k)
      if (!done[k] && klen[k] == L) { out[k] = res[m++]; done[k] = 1; }
  }
out:
  free(sub); free(subfp); free(res); free(done);
  return rc;
}

/* ---- the level loop ---- */

typedef struct {
  const uint8_t *T;
  const uint64_t *st, *len;
  uint64_t c, r;
  uint64_t *fp;
} blockfp_t;

/* fingerprint of every block of the level, by Horner over the block */
static void blocks_fp(void *arg, int t, int K) {
  blockfp_t *a = arg;
  uint64_t lo = a->c * (uint64_t)t / K, hi = a->c * (uint64_t)(t + 1) / K;
  for (uint64_t j = lo; j < hi; ++j) a->fp[j] = phi(a->T, a->st[j], a->len[j], a->r);
}

static double now_ms(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec * 1e3 + ts.tv_nsec * 1e-6;
}

/* Build the tree of T with b1 = leaf * tau^k, on `threads` threads (1..256),
 * Karp-Rabin base r (reduced mod q), fingerprints masked to their low
 * `fp_bits` bits (64 = unmasked; fewer bits force collisions, which byte
 * comparison must absorb).  *err: ORA_OK, ORA_E_INVAL, ORA_E_NOMEM, or
 * ORA_E_LEMMA when a pointer target is not a marked block or pair.
 * stats: NULL, or 4 doubles per level (phase-1 keys, phase-1 ms, phase-2 keys,
 * phase-2 ms) for at least h levels. */
void *ora_build_par(const uint8_t *T, uint64_t n, uint32_t tau, uint32_t leaf, uint64_t b1,
                    int threads, uint64_t r, uint32_t fp_bits, double *stats, int *err) {
  *err = ORA_OK;
  if (tau < 2 || leaf == 0 || b1 == 0 || threads < 1 || threads > 256 || fp_bits == 0 ||
      fp_bits > 64) { *err = ORA_E_INVAL; return NULL; }
  {
    uint64_t b = leaf;
    while (b < b1) b *= tau;
    if (b != b1) { *err = ORA_E_INVAL; return NULL; }
  }
  r %= GQ;
  const uint64_t mask = fp_bits == 64 ? UINT64_MAX : (((uint64_t)1 << fp_bits) - 1);
  uint32_t hmax = 1;
  for (uint64_t b = b1; b > leaf; b /= tau) ++hmax;
  otree *t = calloc(1, sizeof *t);
  if (!t) { *err = ORA_E_NOMEM; return NULL; }
  t->n = n; t->b1 = b1; t->tau = tau; t->leaf = leaf; t->h = hmax;
  t->lv = calloc(hmax, sizeof(olevel));
  if (!t->lv) { free(t); *err = ORA_E_NOMEM; return NULL; }

  uint64_t c = n ? (n + b1 - 1) / b1 : 0;
  uint64_t *st = malloc((c ? c : 1) * 8), *len = malloc((c ? c : 1) * 8);
  if (!st || !len) { free(st); free(len); ora_free_tree(t); *err = ORA_E_NOMEM; return NULL; }
  for (uint64_t j = 0; j < c; ++j) {
    st[j] = j * b1;
    len[j] = (n - st[j] < b1) ? n - st[j] : b1;
  }
  uint64_t b = b1;

  for (uint32_t l = 0; l < hmax; ++l) {
    olevel *Lv = &t->lv[l];
    Lv->b = b; Lv->c = c; Lv->st = st; Lv->len = len;
    Lv->marked = calloc(c ? c : 1, 1);
    if (!Lv->marked) { ora_free_tree(t); *err = ORA_E_NOMEM; return NULL; }
    if (l == hmax - 1) {
      uint64_t tot = 0;
      for (uint64_t j = 0; j < c; ++j) tot += len[j];
      t->leaves = malloc(tot ? tot : 1);
      if (!t->leaves) { ora_free_tree(t); *err = ORA_E_NOMEM; return NULL; }
      uint64_t o = 0;
      for (uint64_t j = 0; j < c; ++j) { memcpy(t->leaves + o, T + st[j], len[j]); o += len[j]; }
      t->leaf_bytes = tot;
      break;
    }
    const uint64_t cc = c ? c : 1;
    uint8_t *adj = calloc(cc, 1);
    uint64_t *rs = malloc(cc * 8), *re = malloc(cc * 8);
    uint64_t *kst = malloc(cc * 8), *klen = malloc(cc * 8), *kj = malloc(cc * 8);
    uint64_t *occ = malloc(cc * 8), *bfp = malloc(cc * 8), *kfp = malloc(cc * 8);
    int rc = ORA_OK;
    if (!adj || !rs || !re || !kst || !klen || !kj || !occ || !bfp || !kfp) {
      rc = ORA_E_NOMEM;
      goto level_done;
    }
    for (uint64_t j = 0; j + 1 < c; ++j) adj[j] = (st[j + 1] == st[j] + len[j]);
    uint64_t R = 0;
    for (uint64_t j = 0; j < c; ++j) {
      if (j == 0 || !adj[j - 1]) { rs[R] = st[j]; re[R] = st[j] + len[j]; ++R; }
      else re[R - 1] = st[j] + len[j];
    }

    /* block fingerprints; a pair's follows from its blocks' by the
     * concatenation rule phi(XY) = phi(X) r^|Y| + phi(Y) */
    double t0 = now_ms();
    {
      blockfp_t a = {T, st, len, c, r, bfp};
      par_for(threads, blocks_fp, &a);
    }
    const uint64_t rb = g_pow(r, b);

    /* first phase: pairs of consecutive blocks */
    uint64_t nk = 0;
    for (uint64_t j = 0; j + 1 < c; ++j)
      if (adj[j]) {
        kst[nk] = st[j];
        klen[nk] = len[j] + len[j + 1];
        kfp[nk] = g_add(g_mul(bfp[j], len[j + 1] == b ? rb : g_pow(r, len[j + 1])), bfp[j + 1]);
        kj[nk] = j;
        ++nk;
      }
    rc = leftmost_mixed(T, kst, klen, kfp, nk, rs, re, R, r, mask, threads, occ);
    if (rc == ORA_E_NOMEM) goto level_done;
    for (uint64_t k = 0; k < nk; ++k)
      if (occ[k] == kst[k]) { Lv->marked[kj[k]] = 1; Lv->marked[kj[k] + 1] = 1; }
    /* blocks with no consecutive neighbour */
    for (uint64_t j = 0; j < c; ++j) {
      int left = (j > 0) && adj[j - 1];
      if (!left && !adj[j]) Lv->marked[j] = 1;
    }
    if (stats) { stats[4 * l] = (double)nk; stats[4 * l + 1] = now_ms() - t0; }

    /* second phase: the unmarked blocks */
    t0 = now_ms();
    nk = 0;
    for (uint64_t j = 0; j < c; ++j)
      if (!Lv->marked[j]) { kst[nk] = st[j]; klen[nk] = len[j]; kfp[nk] = bfp[j]; kj[nk] = j; ++nk; }
    Lv->u = nk;
    Lv->pb = malloc((nk ? nk : 1) * 8);
    Lv->po = malloc((nk ? nk : 1) * 8);
    if (!Lv->pb || !Lv->po) { rc = ORA_E_NOMEM; goto level_done; }
    {
      int e = leftmost_mixed(T, kst, klen, kfp, nk, rs, re, R, r, mask, threads, occ);
      if (e == ORA_E_NOMEM) { rc = e; goto level_done; }
      if (e != ORA_OK) rc = e;
    }
    for (uint64_t k = 0; k < nk; ++k) {
      const uint64_t j = kj[k], p = occ[k];
      uint64_t lo = 0, hi = c;
      while (hi - lo > 1) {
        uint64_t mid = (lo + hi) / 2;
        if (st[mid] <= p) lo = mid; else hi = mid;
      }
      int ok = p >= st[lo] && p < st[lo] + len[lo] && Lv->marked[lo] && p < st[j];
      if (ok && p + len[j] > st[lo] + len[lo])
        ok = lo + 1 < c && adj[lo] && Lv->marked[lo + 1] && p + len[j] <= st[lo + 1] + len[lo + 1];
      if (!ok) rc = ORA_E_LEMMA;
      Lv->pb[k] = lo;
      Lv->po[k] = p - st[lo];
    }
    if (stats) { stats[4 * l + 2] = (double)nk; stats[4 * l + 3] = now_ms() - t0; }

  level_done:
    free(adj); free(rs); free(re); free(kst); free(klen); free(kj); free(occ); free(bfp);
    free(kfp);
    if (rc == ORA_E_NOMEM) { ora_free_tree(t); *err = rc; return NULL; }
    if (rc != ORA_OK) *err = rc;

    /* split the marked blocks into the next level's blocks */
    const uint64_t nb = b / tau;
    uint64_t nc = 0;
    for (uint64_t j = 0; j < c; ++j)
      if (Lv->marked[j]) nc += (len[j] + nb - 1) / nb;
    uint64_t *nst = malloc((nc ? nc : 1) * 8), *nlen = malloc((nc ? nc : 1) * 8);
    if (!nst || !nlen) { free(nst); free(nlen); ora_free_tree(t); *err = ORA_E_NOMEM; return NULL; }
    uint64_t q = 0;
    for (uint64_t j = 0; j < c; ++j) {
      if (!Lv->marked[j]) continue;
      for (uint64_t off = 0; off < len[j]; off += nb) {
        nst[q] = st[j] + off;
        nlen[q] = (len[j] - off < nb) ? len[j] - off : nb;
        ++q;
      }
    }
    st = nst; len = nlen; c = nc; b = nb;
  }
  return t;
}
