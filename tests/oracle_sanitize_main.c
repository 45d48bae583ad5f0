/*
 * Driver for the sanitizer builds of the CPU oracle (tests/test_oracle_sanitize.py):
 * builds trees of small texts with both oracle constructions (the plain
 * definition in every search mode, and the threaded two-phase method with
 * several thread counts and truncated fingerprints), prunes, serializes, and
 * checks that the constructions agree byte for byte.  Exit status 0 when every
 * check holds; the sanitizers abort on any memory, undefined-behaviour or
 * data-race error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

enum { ORA_OK = 0 };
int ora_plan(uint64_t n, uint32_t tau, uint32_t leaf, uint64_t s_hint, uint64_t root_len,
             uint64_t *b1_out, uint32_t *h_out);
void *ora_build(const uint8_t *T, uint64_t n, uint32_t tau, uint32_t leaf, uint64_t b1,
                int exact_split, int search, int *err);
void *ora_build_par(const uint8_t *T, uint64_t n, uint32_t tau, uint32_t leaf, uint64_t b1,
                    int threads, uint64_t r, uint32_t fp_bits, double *stats, int *err);
int ora_prune(void *h, const uint8_t *T);
int ora_serialize(void *h, uint8_t *dst, uint64_t cap, uint64_t *written);
void ora_free(void *h);

static uint8_t *canonical(void *h, uint64_t *len) {
  uint64_t w = 0;
  ora_serialize(h, NULL, 0, &w);
  uint8_t *buf = malloc(w ? w : 1);
  ora_serialize(h, buf, w, &w);
  *len = w;
  return buf;
}

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static uint32_t next(void) {
  rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;
  return (uint32_t)(rng >> 11);
}

int main(void) {
  int failures = 0, cases = 0;
  for (int k = 0; k < 60; ++k) {
    const uint64_t n = next() % 3000;
    const uint32_t sigma = 1 + next() % 4;
    uint8_t *T = malloc(n ? n : 1);
    /* a repetitive text: a random base copied with a few changes */
    const uint64_t base = 1 + next() % 200;
    for (uint64_t i = 0; i < n; ++i)
      T[i] = (uint8_t)(i < base ? 'a' + next() % sigma : T[i - base]);
    for (uint64_t i = 0; i < n / 50; ++i) T[next() % n] = (uint8_t)('a' + next() % sigma);
    const uint32_t tau = 2 + next() % 3, leaf = 1 + next() % 4;
    uint64_t b1;
    uint32_t h;
    if (ora_plan(n, tau, leaf, 1 + next() % 4, 0, &b1, &h) != ORA_OK) return 2;
    int err;
    void *ref = ora_build(T, n, tau, leaf, b1, 1, 0, &err);
    if (!ref || err) return 3;
    uint64_t lr;
    uint8_t *cr = canonical(ref, &lr);
    for (int search = 1; search <= 2; ++search) {
      void *t = ora_build(T, n, tau, leaf, b1, 1, search, &err);
      uint64_t l;
      uint8_t *c = canonical(t, &l);
      failures += err || l != lr || memcmp(c, cr, l) != 0;
      free(c);
      ora_free(t);
    }
    const int threads[3] = {1, 3, 8};
    const uint32_t bits[3] = {64, 5, 12};
    for (int v = 0; v < 3; ++v) {
      double stats[4 * 64];
      void *t = ora_build_par(T, n, tau, leaf, b1, threads[v], 0x1234567 + v, bits[v], stats, &err);
      uint64_t l;
      uint8_t *c = canonical(t, &l);
      failures += err || l != lr || memcmp(c, cr, l) != 0;
      free(c);
      ora_free(t);
      ++cases;
    }
    /* pruning (general split too) */
    void *g = ora_build(T, n, tau, leaf, b1 + (next() % 3), 0, 0, &err);
    if (g) {
      ora_prune(g, T);
      uint64_t l;
      free(canonical(g, &l));
      ora_free(g);
    }
    free(cr);
    ora_free(ref);
    free(T);
  }
  printf("%d threaded cases, %d failures\n", cases, failures);
  return failures ? 1 : 0;
}
