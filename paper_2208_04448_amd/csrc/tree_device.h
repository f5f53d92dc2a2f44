// Device-side leaf lookup shared by the kernels that locate voxels in a built
// tree (random access, topology patches, archive decoding).
#pragma once
#include "nvdb_internal.h"

namespace nvdb {

// Canonical order of two leaf origins (both multiples of 8): level-2 origin
// (arithmetic shifts floor negative coordinates), then the level-1 slot n2,
// then the leaf slot n1.
__device__ __forceinline__ bool leaf_before(const int4& a, const int4& b) {
  if ((a.x >> 12) != (b.x >> 12)) return (a.x >> 12) < (b.x >> 12);
  if ((a.y >> 12) != (b.y >> 12)) return (a.y >> 12) < (b.y >> 12);
  if ((a.z >> 12) != (b.z >> 12)) return (a.z >> 12) < (b.z >> 12);
  const int an2 = (((a.x >> 7) & 31) << 10) | (((a.y >> 7) & 31) << 5) | ((a.z >> 7) & 31);
  const int bn2 = (((b.x >> 7) & 31) << 10) | (((b.y >> 7) & 31) << 5) | ((b.z >> 7) & 31);
  if (an2 != bn2) return an2 < bn2;
  const int an1 = (((a.x >> 3) & 15) << 8) | (((a.y >> 3) & 15) << 4) | ((a.z >> 3) & 15);
  const int bn1 = (((b.x >> 3) & 15) << 8) | (((b.y >> 3) & 15) << 4) | ((b.z >> 3) & 15);
  return an1 < bn1;
}

struct QueryTree {
  const int4* leaf_o;
  const uint64_t* leaf_mask;
  int64_t n_leaf;
};

// Canonical order of level-1 nodes: level-2 origin (x, y, z), then the slot n2.
__device__ __forceinline__ bool l1_before(int4 a, int4 b) {
  const int ax = a.x & ~4095, ay = a.y & ~4095, az = a.z & ~4095;
  const int bx = b.x & ~4095, by = b.y & ~4095, bz = b.z & ~4095;
  if (ax != bx) return ax < bx;
  if (ay != by) return ay < by;
  if (az != bz) return az < bz;
  const int na = (((a.x >> 7) & 31) << 10) | (((a.y >> 7) & 31) << 5) | ((a.z >> 7) & 31);
  const int nb = (((b.x >> 7) & 31) << 10) | (((b.y >> 7) & 31) << 5) | ((b.z >> 7) & 31);
  return na < nb;
}
// First index among the n canonical level-1 origins that is not before o (o itself
// when that node exists).
__device__ __forceinline__ int64_t lower_l1(const int4* l1_o, int64_t n, int4 o) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (l1_before(l1_o[mid], o)) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Index of the leaf of t with origin o, or -1.
__device__ __forceinline__ int64_t find_leaf(const QueryTree& t, const int4& o) {
  int64_t a = 0, b = t.n_leaf;
  while (a < b) {
    const int64_t m = (a + b) >> 1;
    if (leaf_before(t.leaf_o[m], o)) a = m + 1;
    else b = m;
  }
  if (a < t.n_leaf) {
    const int4 f = t.leaf_o[a];
    if (f.x == o.x && f.y == o.y && f.z == o.z) return a;
  }
  return -1;
}

}  // namespace nvdb
