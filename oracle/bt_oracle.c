/*
 * Block-tree oracle: a plain, slow, obviously correct CPU construction of the
 * block tree of Belazzougui et al. as restated in "Practical Parallel Block
 * Tree Construction: First Results" (Clausecker, Kurpicz, Palanga).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the GPU library.
 *
 * What it computes (Section 4, block-tree definition; Section 4.1, the two
 * phases), 0-based:
 *   level 1   blocks start at 0, b1, 2*b1, ... < n; the last one may be short.
 *   level l   (while the block length b exceeds leaf_len)
 *     adj(j)      block j+1 exists and starts where block j ends
 *     pair rule   for adj(j): X = B_j B_{j+1}; if the leftmost occurrence of X
 *                 in T starts at st_j, mark j and j+1          (Section 4)
 *     isolated    a block with no adjacent neighbour on either side is marked
 *     pointers    each unmarked j points at (t, off): p = leftmost occurrence
 *                 of B_j in T, t = the level block containing p, off = p-st_t
 *                 (Section 4, pointer to the pair holding the leftmost
 *                 occurrence, plus its offset; Section 4.1, second phase)
 *     split       each marked block, in order, gets children of length
 *                 b/tau (exact mode) or ceil(b/tau) (general mode, used by
 *                 the worked example of Figure 1), clipped at its own end
 *   last level  the blocks are stored explicitly as leaf bytes (Section 4,
 *               the stopping rule |B| in Theta(log_sigma n)).
 * Leftmost occurrences are found by direct search: memmem (default) or a
 * literal double loop.  No fingerprints, no hashing.
 *
 * A second search scope restricts candidate occurrences to windows that lie
 * inside runs of consecutive blocks of the current level ("leftmost occurrence
 * on this level", Section 4); tests assert both scopes give the same tree.
 *
 * Optional pruning (Section 4.1) is a separate pass over a built tree; its
 * reading is stated where it is defined.
 *
 * Also here: prefix Karp-Rabin fingerprints mod 2^61-1 by Horner's rule
 * (Section 2, the definition of phi), and counted-prefix access/rank/select
 * (Section 1, query definitions), each a plain definition.
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "ora_tree.h"

/* ---- level plan (build parameters; see the header for the policy) ---- */

/* Largest k >= 0 with leaf * tau^k <= lim (k = 0 when lim < leaf). */
static uint32_t max_pow_le(uint64_t leaf, uint32_t tau, uint64_t lim, uint64_t *blen) {
  uint32_t k = 0;
  uint64_t b = leaf;
  while (b <= lim / tau && b * tau <= lim) { b *= tau; ++k; }
  *blen = b;
  return k;
}

int ora_plan(uint64_t n, uint32_t tau, uint32_t leaf, uint64_t s_hint,
             uint64_t root_len, uint64_t *b1_out, uint32_t *h_out) {
  if (tau < 2 || leaf == 0) return ORA_E_INVAL;
  uint64_t b;
  uint32_t k;
  if (root_len) {
    b = leaf; k = 0;
    while (b < root_len) {
      if (b > UINT64_MAX / tau) return ORA_E_INVAL;
      b *= tau; ++k;
    }
    if (b != root_len) return ORA_E_INVAL;
  } else {
    uint64_t s = s_hint ? s_hint : 1;
    k = max_pow_le(leaf, tau, n / s, &b);
  }
  *b1_out = b;
  *h_out = k + 1;
  return ORA_OK;
}

/* ---- leftmost occurrence by direct search ---- */

/* First p <= st with T[p..p+L) == T[st..st+L), searching all of T.
 * mode 0: memmem; mode 1: literal double loop. */
static uint64_t leftmost_whole(const uint8_t *T, uint64_t st, uint64_t L, int mode) {
  if (L == 0) return 0;
  if (mode == 0) {
    const void *r = memmem(T, st + L, T + st, L);
    return (uint64_t)((const uint8_t *)r - T);
  }
  for (uint64_t p = 0; p <= st; ++p) {
    uint64_t k = 0;
    while (k < L && T[p + k] == T[st + k]) ++k;
    if (k == L) return p;
  }
  return st;
}

/* Same, but only windows lying inside one run of consecutive level blocks.
 * runs are [rs[r], re[r]) in increasing order. */
static uint64_t leftmost_in_runs(const uint8_t *T, uint64_t st, uint64_t L,
                                 const uint64_t *rs, const uint64_t *re, uint64_t R) {
  for (uint64_t r = 0; r < R; ++r) {
    if (rs[r] > st) break;
    uint64_t end = re[r];
    if (end > st + L) end = st + L;
    if (end < rs[r] + L) continue;
    const void *hit = memmem(T + rs[r], end - rs[r], T + st, L);
    if (hit) return (uint64_t)((const uint8_t *)hit - T);
  }
  return UINT64_MAX; /* unreachable: the block itself lies in a run */
}

/* ---- construction ---- */

void ora_free_tree(otree *t) {
  if (!t) return;
  if (t->lv) {
    for (uint32_t l = 0; l < t->h; ++l) {
      free(t->lv[l].st); free(t->lv[l].len); free(t->lv[l].marked);
      free(t->lv[l].pb); free(t->lv[l].po);
    }
    free(t->lv);
  }
  free(t->leaves);
  free(t);
}

/* Build the tree.  exact_split: 1 requires b1 = leaf*tau^k and splits into
 * b/tau; 0 splits into ceil(b/tau) (Figure 1 style).  search: 0 memmem over T,
 * 1 literal double loop over T, 2 memmem restricted to level runs. */
void *ora_build(const uint8_t *T, uint64_t n, uint32_t tau, uint32_t leaf,
                uint64_t b1, int exact_split, int search, int *err) {
  *err = ORA_OK;
  if (tau < 2 || leaf == 0 || b1 == 0) { *err = ORA_E_INVAL; return NULL; }
  uint32_t hmax = 1;
  for (uint64_t b = b1; b > leaf; b = exact_split ? b / tau : (b + tau - 1) / tau) ++hmax;
  if (exact_split) {
    uint64_t b = leaf;
    while (b < b1) b *= tau;
    if (b != b1) { *err = ORA_E_INVAL; return NULL; }
  }
  otree *t = calloc(1, sizeof *t);
  if (!t) { *err = ORA_E_NOMEM; return NULL; }
  t->n = n; t->b1 = b1; t->tau = tau; t->leaf = leaf; t->h = hmax;
  t->lv = calloc(hmax, sizeof(olevel));
  if (!t->lv) { free(t); *err = ORA_E_NOMEM; return NULL; }

  /* level 1 */
  uint64_t c = n ? (n + b1 - 1) / b1 : 0;
  uint64_t *st = malloc((c ? c : 1) * sizeof(uint64_t));
  uint64_t *len = malloc((c ? c : 1) * sizeof(uint64_t));
  if (!st || !len) { free(st); free(len); ora_free_tree(t); *err = ORA_E_NOMEM; return NULL; }
  for (uint64_t j = 0; j < c; ++j) {
    st[j] = j * b1;
    len[j] = (n - st[j] < b1) ? n - st[j] : b1;
  }
  uint64_t b = b1;

  for (uint32_t l = 0; l < hmax; ++l) {
    olevel *L = &t->lv[l];
    L->b = b; L->c = c; L->st = st; L->len = len;
    L->marked = calloc(c ? c : 1, 1);
    if (!L->marked) { ora_free_tree(t); *err = ORA_E_NOMEM; return NULL; }
    if (l == hmax - 1) {
      /* leaves: every block of the last level, stored explicitly */
      uint64_t tot = 0;
      for (uint64_t j = 0; j < c; ++j) tot += len[j];
      t->leaves = malloc(tot ? tot : 1);
      if (!t->leaves) { ora_free_tree(t); *err = ORA_E_NOMEM; return NULL; }
      uint64_t o = 0;
      for (uint64_t j = 0; j < c; ++j) { memcpy(t->leaves + o, T + st[j], len[j]); o += len[j]; }
      t->leaf_bytes = tot;
      break;
    }
    uint8_t *adj = calloc(c ? c : 1, 1);
    if (!adj) { ora_free_tree(t); *err = ORA_E_NOMEM; return NULL; }
    for (uint64_t j = 0; j + 1 < c; ++j) adj[j] = (st[j + 1] == st[j] + len[j]);

    /* runs of consecutive blocks, for the restricted search scope */
    uint64_t R = 0, *rs = NULL, *re = NULL;
    if (search == 2) {
      rs = malloc((c ? c : 1) * sizeof(uint64_t));
      re = malloc((c ? c : 1) * sizeof(uint64_t));
      if (!rs || !re) { free(adj); free(rs); free(re); ora_free_tree(t); *err = ORA_E_NOMEM; return NULL; }
      for (uint64_t j = 0; j < c; ++j) {
        if (j == 0 || !adj[j - 1]) { rs[R] = st[j]; re[R] = st[j] + len[j]; ++R; }
        else re[R - 1] = st[j] + len[j];
      }
    }
#define LEFTMOST(s_, L_) (search == 2 ? leftmost_in_runs(T, (s_), (L_), rs, re, R) \
                                      : leftmost_whole(T, (s_), (L_), search))
    /* first phase: pairs of consecutive blocks */
    for (uint64_t j = 0; j + 1 < c; ++j) {
      if (!adj[j]) continue;
      uint64_t p = LEFTMOST(st[j], len[j] + len[j + 1]);
      if (p == st[j]) { L->marked[j] = 1; L->marked[j + 1] = 1; }
    }
    /* blocks with no consecutive neighbour */
    for (uint64_t j = 0; j < c; ++j) {
      int left = (j > 0) && adj[j - 1];
      if (!left && !adj[j]) L->marked[j] = 1;
    }
    /* second phase: pointers of unmarked blocks */
    uint64_t u = 0;
    for (uint64_t j = 0; j < c; ++j) u += !L->marked[j];
    L->u = u;
    L->pb = malloc((u ? u : 1) * sizeof(uint64_t));
    L->po = malloc((u ? u : 1) * sizeof(uint64_t));
    if (!L->pb || !L->po) { free(adj); free(rs); free(re); ora_free_tree(t); *err = ORA_E_NOMEM; return NULL; }
    uint64_t k = 0;
    for (uint64_t j = 0; j < c; ++j) {
      if (L->marked[j]) continue;
      uint64_t p = LEFTMOST(st[j], len[j]);
      /* the block of this level containing p (blocks are sorted by start) */
      uint64_t lo = 0, hi = c;
      while (hi - lo > 1) {
        uint64_t mid = (lo + hi) / 2;
        if (st[mid] <= p) lo = mid; else hi = mid;
      }
      uint64_t tt = lo;
      /* the occurrence must lie in marked block tt, or in the marked
       * consecutive pair (tt, tt+1) */
      int ok = p >= st[tt] && p < st[tt] + len[tt] && L->marked[tt] && p < st[j];
      if (ok && p + len[j] > st[tt] + len[tt])
        ok = tt + 1 < c && adj[tt] && L->marked[tt + 1] &&
             p + len[j] <= st[tt + 1] + len[tt + 1];
      if (!ok) *err = ORA_E_LEMMA;
      L->pb[k] = tt;
      L->po[k] = p - st[tt];
      ++k;
    }
#undef LEFTMOST
    free(adj); free(rs); free(re);

    /* split marked blocks into the next level's blocks */
    uint64_t nb = exact_split ? b / tau : (b + tau - 1) / tau;
    uint64_t nc = 0;
    for (uint64_t j = 0; j < c; ++j)
      if (L->marked[j]) nc += (len[j] + nb - 1) / nb;
    uint64_t *nst = malloc((nc ? nc : 1) * sizeof(uint64_t));
    uint64_t *nlen = malloc((nc ? nc : 1) * sizeof(uint64_t));
    if (!nst || !nlen) { free(nst); free(nlen); ora_free_tree(t); *err = ORA_E_NOMEM; return NULL; }
    uint64_t q = 0;
    for (uint64_t j = 0; j < c; ++j) {
      if (!L->marked[j]) continue;
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

/* ---- optional pruning (Section 4.1, the optional third phase) ----
 *
 * Marked blocks that no pointer targets are turned into pointers.  Reading
 * (the paper gives the rule in one paragraph, without an order):
 *   - internal levels are visited from the deepest up; within a level, blocks
 *     from right to left (every pointer targets blocks to the left of its own,
 *     so a block is judged after every pointer that can target it);
 *   - a marked block j becomes a pointer when (i) no pointer of its level
 *     targets it, counting those made by pruning, (ii) none of its children is
 *     marked (children on the leaf level are leaves), and (iii) the leftmost
 *     occurrence p of B_j among the windows inside runs of consecutive level
 *     blocks ends at or before st_j (an occurrence that reaches into B_j would
 *     need B_j to stay marked), and (iv) that occurrence lies in one block or
 *     in two consecutive ones (always so when every block but a text's last
 *     has full length);
 *   - it then points at (t, p - st_t), t the block holding p, marks t (and t+1
 *     when the occurrence spills into it) as targeted, and its children leave
 *     the level below; the children's own pointers go with them, and levels
 *     already visited are not visited again.
 * T is the text the tree was built from. */
int ora_prune(void *hdl, const uint8_t *T) {
  otree *t = hdl;
  int rc = ORA_OK;
  for (int l = (int)t->h - 2; l >= 0; --l) {
    olevel *L = &t->lv[l], *C = &t->lv[l + 1];
    const int child_is_leaf = (l + 1 == (int)t->h - 1);
    const uint64_t c = L->c, cc = C->c;
    uint8_t *adj = calloc(c ? c : 1, 1), *tgt = calloc(c ? c : 1, 1);
    uint8_t *gone = calloc(cc ? cc : 1, 1);
    uint64_t *rs = malloc((c ? c : 1) * 8), *re = malloc((c ? c : 1) * 8);
    uint64_t *qb = malloc((c ? c : 1) * 8), *qo = malloc((c ? c : 1) * 8);
    uint64_t *cf = malloc((c + 1) * 8);
    if (!adj || !tgt || !gone || !rs || !re || !qb || !qo || !cf) {
      free(adj); free(tgt); free(gone); free(rs); free(re); free(qb); free(qo); free(cf);
      return ORA_E_NOMEM;
    }
    uint64_t R = 0;
    for (uint64_t j = 0; j < c; ++j) {
      if (j + 1 < c) adj[j] = (L->st[j + 1] == L->st[j] + L->len[j]);
      if (j == 0 || !adj[j - 1]) { rs[R] = L->st[j]; re[R] = L->st[j] + L->len[j]; ++R; }
      else re[R - 1] = L->st[j] + L->len[j];
    }
    /* every unmarked block's pointer, indexed by block, and what it targets */
    for (uint64_t j = 0, k = 0; j < c; ++j) {
      if (L->marked[j]) continue;
      qb[j] = L->pb[k]; qo[j] = L->po[k]; ++k;
      tgt[qb[j]] = 1;
      if (qo[j] + L->len[j] > L->len[qb[j]]) tgt[qb[j] + 1] = 1;
    }
    /* children: marked blocks, in order, own consecutive ranges of the level below */
    cf[0] = 0;
    for (uint64_t j = 0; j < c; ++j)
      cf[j + 1] = cf[j] + (L->marked[j] ? (L->len[j] + C->b - 1) / C->b : 0);
    uint64_t npruned = 0;
    for (uint64_t j = c; j-- > 0;) {
      if (!L->marked[j] || tgt[j]) continue;
      int inner = 0;
      if (!child_is_leaf)
        for (uint64_t i = cf[j]; i < cf[j + 1]; ++i) inner |= C->marked[i];
      if (inner) continue;
      const uint64_t p = leftmost_in_runs(T, L->st[j], L->len[j], rs, re, R);
      if (p + L->len[j] > L->st[j]) continue;
      uint64_t lo = 0, hi = c;
      while (hi - lo > 1) {
        uint64_t mid = (lo + hi) / 2;
        if (L->st[mid] <= p) lo = mid; else hi = mid;
      }
      const int spill = p + L->len[j] > L->st[lo] + L->len[lo];
      /* (iv) a pointer names one block or a consecutive pair; a split into
       * ceil(b/tau) can leave a short block inside a run, and an occurrence
       * across three blocks keeps the block marked */
      if (spill && (lo + 1 >= c || !adj[lo] ||
                    p + L->len[j] > L->st[lo + 1] + L->len[lo + 1])) continue;
      if (!L->marked[lo] || (spill && !L->marked[lo + 1])) { rc = ORA_E_LEMMA; continue; }
      L->marked[j] = 0;
      qb[j] = lo; qo[j] = p - L->st[lo];
      tgt[lo] = 1;
      if (spill) tgt[lo + 1] = 1;
      for (uint64_t i = cf[j]; i < cf[j + 1]; ++i) gone[i] = 1;
      ++npruned;
    }
    if (npruned) {
      /* this level's pointer arrays, in block order */
      uint64_t u = L->u + npruned;
      uint64_t *pb = malloc(u * 8), *po = malloc(u * 8);
      if (!pb || !po) { rc = ORA_E_NOMEM; free(pb); free(po); }
      else {
        for (uint64_t j = 0, k = 0; j < c; ++j)
          if (!L->marked[j]) { pb[k] = qb[j]; po[k] = qo[j]; ++k; }
        free(L->pb); free(L->po);
        L->pb = pb; L->po = po; L->u = u;
      }
      /* the level below loses the children of pruned blocks */
      uint64_t *nidx = malloc((cc ? cc : 1) * 8);
      if (!nidx) rc = ORA_E_NOMEM;
      else {
        uint64_t kept = 0;
        for (uint64_t i = 0; i < cc; ++i) { nidx[i] = kept; kept += !gone[i]; }
        if (child_is_leaf) {
          uint64_t src = 0, dst = 0;
          for (uint64_t i = 0; i < cc; ++i) {
            if (!gone[i]) memmove(t->leaves + dst, t->leaves + src, C->len[i]);
            dst += gone[i] ? 0 : C->len[i];
            src += C->len[i];
          }
          t->leaf_bytes = dst;
        } else {
          uint64_t k = 0, w = 0;
          for (uint64_t i = 0; i < cc; ++i) {
            if (C->marked[i]) continue;
            if (!gone[i]) { C->pb[w] = nidx[C->pb[k]]; C->po[w] = C->po[k]; ++w; }
            ++k;
          }
          C->u = w;
        }
        for (uint64_t i = 0; i < cc; ++i)
          if (!gone[i]) {
            C->st[nidx[i]] = C->st[i]; C->len[nidx[i]] = C->len[i];
            C->marked[nidx[i]] = C->marked[i];
          }
        C->c = kept;
        free(nidx);
      }
    }
    free(adj); free(tgt); free(gone); free(rs); free(re); free(qb); free(qo); free(cf);
    if (rc == ORA_E_NOMEM) return rc;
  }
  return rc;
}

void ora_free(void *h) { ora_free_tree((otree *)h); }

int ora_tree_info(void *h, uint64_t *n, uint32_t *height, uint64_t *b1, uint64_t *leaf_bytes) {
  otree *t = h;
  *n = t->n; *height = t->h; *b1 = t->b1; *leaf_bytes = t->leaf_bytes;
  return ORA_OK;
}

int ora_level_info(void *h, uint32_t level, uint64_t *b, uint64_t *c, uint64_t *u) {
  otree *t = h;
  if (level < 1 || level > t->h) return ORA_E_INVAL;
  olevel *L = &t->lv[level - 1];
  *b = L->b; *c = L->c; *u = L->u;
  return ORA_OK;
}

/* Copy a level's arrays; any destination may be NULL. */
int ora_level_copy(void *h, uint32_t level, uint8_t *marked, uint64_t *st,
                   uint64_t *len, uint64_t *pb, uint64_t *po) {
  otree *t = h;
  if (level < 1 || level > t->h) return ORA_E_INVAL;
  olevel *L = &t->lv[level - 1];
  if (marked) memcpy(marked, L->marked, L->c);
  if (st) memcpy(st, L->st, L->c * sizeof(uint64_t));
  if (len) memcpy(len, L->len, L->c * sizeof(uint64_t));
  if (pb && L->u) memcpy(pb, L->pb, L->u * sizeof(uint64_t));
  if (po && L->u) memcpy(po, L->po, L->u * sizeof(uint64_t));
  return ORA_OK;
}

int ora_leaves(void *h, uint8_t *out) {
  otree *t = h;
  if (t->leaf_bytes) memcpy(out, t->leaves, t->leaf_bytes);
  return ORA_OK;
}

/* ---- canonical serialisation (format documented with the C ABI) ---- */

static uint64_t put(uint8_t *dst, uint64_t cap, uint64_t at, const void *src, uint64_t k) {
  if (dst && at + k <= cap) memcpy(dst + at, src, k);
  return at + k;
}

int ora_serialize(void *h, uint8_t *dst, uint64_t cap, uint64_t *written) {
  otree *t = h;
  uint64_t at = 0;
  uint32_t zero = 0;
  at = put(dst, cap, at, "BTv1", 4);
  at = put(dst, cap, at, &t->n, 8);
  at = put(dst, cap, at, &t->tau, 4);
  at = put(dst, cap, at, &t->leaf, 4);
  at = put(dst, cap, at, &t->b1, 8);
  at = put(dst, cap, at, &t->h, 4);
  at = put(dst, cap, at, &zero, 4);
  for (uint32_t l = 0; l + 1 < t->h; ++l) {
    olevel *L = &t->lv[l];
    at = put(dst, cap, at, &L->b, 8);
    at = put(dst, cap, at, &L->c, 8);
    for (uint64_t w = 0; w < (L->c + 63) / 64; ++w) {
      uint64_t word = 0;
      for (uint64_t k = 0; k < 64 && w * 64 + k < L->c; ++k)
        if (L->marked[w * 64 + k]) word |= (uint64_t)1 << k;
      at = put(dst, cap, at, &word, 8);
    }
    at = put(dst, cap, at, &L->u, 8);
    for (uint64_t k = 0; k < L->u; ++k) at = put(dst, cap, at, &L->pb[k], 8);
    for (uint64_t k = 0; k < L->u; ++k) at = put(dst, cap, at, &L->po[k], 8);
  }
  olevel *Lh = &t->lv[t->h - 1];
  at = put(dst, cap, at, &Lh->b, 8);
  at = put(dst, cap, at, &Lh->c, 8);
  at = put(dst, cap, at, &t->leaf_bytes, 8);
  at = put(dst, cap, at, t->leaves, t->leaf_bytes);
  uint64_t pad = (8 - (t->leaf_bytes & 7)) & 7;
  uint64_t zeros = 0;
  at = put(dst, cap, at, &zeros, pad);
  *written = at;
  return (dst && at > cap) ? ORA_E_INVAL : ORA_OK;
}

/* ---- Karp-Rabin prefix fingerprints (Section 2, phi) ---- */

#define P61 ((((uint64_t)1) << 61) - 1)

/* P[0] = 0, P[i+1] = (P[i]*x + T[i]) mod (2^61-1); x must be < 2^61-1. */
int ora_prefix_fp(const uint8_t *T, uint64_t n, uint64_t x, uint64_t *P) {
  if (x >= P61) return ORA_E_INVAL;
  unsigned __int128 h = 0;
  P[0] = 0;
  for (uint64_t i = 0; i < n; ++i) {
    h = (h * x + T[i]) % P61;
    P[i + 1] = (uint64_t)h;
  }
  return ORA_OK;
}

/* phi of T[s..s+L) by Horner's rule over the window itself. */
uint64_t ora_window_fp(const uint8_t *T, uint64_t s, uint64_t L, uint64_t x) {
  unsigned __int128 h = 0;
  for (uint64_t k = 0; k < L; ++k) h = (h * x + T[s + k]) % P61;
  return (uint64_t)h;
}

/* ---- counted-prefix queries (Section 1, access/rank/select) ---- */

/* access(i) = T[i]; out-of-range -> 0 (flagged by returning ORA_E_INVAL). */
int ora_access(const uint8_t *T, uint64_t n, const uint64_t *pos, uint64_t m, uint8_t *out) {
  int rc = ORA_OK;
  for (uint64_t q = 0; q < m; ++q) {
    if (pos[q] < n) out[q] = T[pos[q]];
    else { out[q] = 0; rc = ORA_E_INVAL; }
  }
  return rc;
}

typedef struct { uint64_t key; uint64_t idx; } kv;
static int cmp_kv(const void *a, const void *b) {
  const kv *x = a, *y = b;
  return (x->key > y->key) - (x->key < y->key);
}

/* rank(c, i) = #{ j < i : T[j] = c }, i in [0, n]; otherwise UINT64_MAX.
 * Queries are answered in one left-to-right sweep over T, in position order. */
int ora_rank(const uint8_t *T, uint64_t n, const uint8_t *cs, const uint64_t *pos,
             uint64_t m, uint64_t *out) {
  kv *ord = malloc((m ? m : 1) * sizeof(kv));
  if (!ord) return ORA_E_NOMEM;
  for (uint64_t q = 0; q < m; ++q) { ord[q].key = pos[q]; ord[q].idx = q; }
  qsort(ord, m, sizeof(kv), cmp_kv);
  uint64_t cnt[256] = {0};
  uint64_t i = 0;
  for (uint64_t r = 0; r < m; ++r) {
    uint64_t q = ord[r].idx;
    if (pos[q] > n) { out[q] = UINT64_MAX; continue; }
    while (i < pos[q]) { cnt[T[i]]++; ++i; }
    out[q] = cnt[cs[q]];
  }
  free(ord);
  return ORA_OK;
}

/* select(c, k) = the position j with T[j] = c and #{ j' < j : T[j'] = c } = k-1,
 * for k >= 1; UINT64_MAX when k = 0 or c occurs fewer than k times. */
int ora_select(const uint8_t *T, uint64_t n, const uint8_t *cs, const uint64_t *ks,
               uint64_t m, uint64_t *out) {
  kv *ord = malloc((m ? m : 1) * sizeof(kv));
  if (!ord) return ORA_E_NOMEM;
  for (uint64_t q = 0; q < m; ++q) {
    /* sort by (character, k); k is below 2^56 for any text that fits memory */
    uint64_t k = ks[q] > (((uint64_t)1 << 56) - 1) ? (((uint64_t)1 << 56) - 1) : ks[q];
    ord[q].key = ((uint64_t)cs[q] << 56) | k;
    ord[q].idx = q;
    out[q] = UINT64_MAX;
  }
  qsort(ord, m, sizeof(kv), cmp_kv);
  /* per character, the first query in sorted order */
  uint64_t head[257];
  for (int c = 0; c <= 256; ++c) head[c] = m;
  for (uint64_t r = m; r-- > 0;) head[ord[r].key >> 56] = r;
  uint64_t next[256], cnt[256] = {0};
  for (int c = 0; c < 256; ++c) next[c] = head[c];
  for (uint64_t j = 0; j < n; ++j) {
    uint8_t c = T[j];
    cnt[c]++;
    while (next[c] < m && (ord[next[c]].key >> 56) == c &&
           (ord[next[c]].key & ((((uint64_t)1) << 56) - 1)) <= cnt[c]) {
      uint64_t q = ord[next[c]].idx;
      if (ks[q] == cnt[c]) out[q] = j;
      next[c]++;
    }
  }
  free(ord);
  return ORA_OK;
}
