/*
 * The oracle's in-memory block tree, shared by its two constructions: the
 * plain definition (bt_oracle.c) and the paper's own method on host threads
 * (bt_par.c).  TEST INFRASTRUCTURE ONLY; nothing in the GPU library includes
 * this file.
 */
#ifndef ORA_TREE_H
#define ORA_TREE_H
#include <stdint.h>

enum { ORA_OK = 0, ORA_E_INVAL = -1, ORA_E_NOMEM = -2, ORA_E_LEMMA = -3 };

typedef struct {
  uint64_t b, c, u;     /* block length, #blocks, #unmarked */
  uint64_t *st, *len;   /* block starts and lengths (c each) */
  uint8_t *marked;      /* c bytes, 0/1 */
  uint64_t *pb, *po;    /* pointers of unmarked blocks in block order (u each) */
} olevel;

typedef struct {
  uint64_t n, b1;
  uint32_t tau, leaf, h;
  olevel *lv;           /* h levels; the last holds the leaves */
  uint8_t *leaves;      /* concatenated leaf bytes */
  uint64_t leaf_bytes;
} otree;

void ora_free_tree(otree *t);

#endif
