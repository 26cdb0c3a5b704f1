// Per-row column index of a dynamic matrix (device side).
//
// Section 4 gives every row of the dynamic structure a hash table from
// column to position, so that an update finds its entry in constant time.
// Rows here are slot ranges in no column order; the index adds, per row, an
// open-addressing table (linear probing, 2 * length + 16 slots when built,
// a column's first slot by multiplying its hash into the table size) whose
// slots hold (position in the row << 32 | column), all ones when empty; a
// deleted entry leaves a tombstone (column field 0xfffffffe) that lookups
// pass over.  Tables live in one pool per matrix and are taken from its top.
//
// A row's table is usable only while stamp[i] == gen.  The apply keeps it:
// overwrites in place change nothing, inserts are recorded, deletions leave
// tombstones, entries moved into holes get their new position, and a row
// moved as a whole keeps its positions.  A table whose slots in use (live
// entries and tombstones) would pass 3/4 of its size is dropped instead.
// Writers that reorder a row otherwise (a recomputed row, a row compacted
// into new space) invalidate it: per row by clearing the stamp, or all rows
// at once by advancing gen on the host.  Invalid rows are rebuilt from the
// row itself before the next use.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

constexpr uint64_t IX_EMPTY = ~0ull;
constexpr uint64_t IX_TOMB = ~0ull - 1;

struct RowIx {
  uint64_t* tab = nullptr;  // null: the matrix has no index
  int64_t* off = nullptr;   // per row: first slot of its table
  int32_t* sz = nullptr;    // per row: table size
  int32_t* used = nullptr;  // per row: slots taken (entries and tombstones)
  uint32_t* stamp = nullptr;
  unsigned long long* top = nullptr;  // device: first free slot of the pool
  int64_t cap = 0;
  uint32_t gen = 1;
};

__device__ inline uint32_t ix_hash(int32_t c) {
  uint32_t x = (uint32_t)c;
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ inline bool ix_valid(const RowIx& X, int32_t i) { return X.tab && X.stamp[i] == X.gen; }

// first slot of column c in a table of n slots, and the slot after h
__device__ inline uint32_t ix_home(int32_t c, uint32_t n) {
  return (uint32_t)(((uint64_t)ix_hash(c) * n) >> 32);
}
__device__ inline uint32_t ix_next(uint32_t h, uint32_t n) { return h + 1 == n ? 0u : h + 1; }

// position of column c in a row whose table is t (n slots), or -1
__device__ inline int32_t ix_find(const uint64_t* t, uint32_t n, int32_t c) {
  uint32_t h = ix_home(c, n);
  for (;;) {
    const uint64_t e = t[h];
    if ((uint32_t)e == (uint32_t)c) return (int32_t)(e >> 32);
    if (e == IX_EMPTY) return -1;
    h = ix_next(h, n);
  }
}

__device__ inline int32_t ix_lookup(const RowIx& X, int32_t i, int32_t c) {
  return ix_find(X.tab + X.off[i], (uint32_t)X.sz[i], c);
}

// record (column c at position p); the column must not be in the table
__device__ inline void ix_put(uint64_t* t, uint32_t n, int32_t c, int32_t p) {
  const uint64_t v = ((uint64_t)(uint32_t)p << 32) | (uint64_t)(uint32_t)c;
  uint32_t h = ix_home(c, n);
  while (atomicCAS((unsigned long long*)&t[h], (unsigned long long)IX_EMPTY, (unsigned long long)v) !=
         (unsigned long long)IX_EMPTY)
    h = ix_next(h, n);
}

// table slot holding column c, or -1
__device__ inline int32_t ix_slot(const uint64_t* t, uint32_t n, int32_t c) {
  uint32_t h = ix_home(c, n);
  for (;;) {
    const uint64_t e = t[h];
    if ((uint32_t)e == (uint32_t)c) return (int32_t)h;
    if (e == IX_EMPTY) return -1;
    h = ix_next(h, n);
  }
}

// The table stays usable after `add` more slots are taken while at most 3/4
// of it is in use.
__device__ inline bool ix_fits(const RowIx& X, int32_t i, int32_t add) {
  return ((int64_t)X.used[i] + add) * 4 <= (int64_t)X.sz[i] * 3;
}
