// Sparse domain decomposition (NeuralVDB Sec. 3.4, eq. moe).
//
// Index space is cut into a regular grid of cubic cells of edge S; the widened
// box of cell c is its core [o + cS, o + (c+1)S) grown by a halo of h voxels on
// every side.  Each kept cell has an expert network normalised to its widened
// box, and a voxel's value is the average of the experts whose box holds it,
// weighted by clamped-tent gates (product over the axes of
// min(t, S + 2h - t, 2h) / 2h, t the distance of the voxel centre from the
// box's lower face).  With S >= 2h a voxel meets at most two cells per axis,
// so at most eight experts.
//
// The blended decode routes every (voxel, expert) pair into a per-expert bucket
// of normalised coordinates, runs each expert's forward pass over its bucket,
// scatters the outputs into eight slots per voxel, and blends the slots in a
// fixed order (deterministic: bucket order never reaches the sums).  Slot j of
// item i sits at j n + i: eight planes of n slots, so that one expert's outputs
// for consecutive items land side by side and the blend reads each plane
// coalesced.
#include <algorithm>
#include <cfloat>
#include <climits>
#include <vector>

#include "nvdb_internal.h"

namespace nvdb {

namespace {

// Where the items of a blended decode come from.
struct ItemSrc {
  const int4* org;      // leaf origins, or level-1 origins (leaf-slot items)
  const uint32_t* key;  // voxel keys (voxel items), active-tile keys (l1), or null
  int l1;               // 1: leaf slots of the level-1 nodes
};

// Floor division in 64 bits: p - o can leave the int32 range for far grid origins.
__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t s) { return a >= 0 ? a / s : -((-a + s - 1) / s); }

__device__ __forceinline__ int3 voxel_of(const int4* __restrict__ leaf_o, uint32_t key) {
  const int4 o = leaf_o[key >> 9];
  const uint32_t n0 = key & 511u;
  return make_int3(o.x + (int)(n0 >> 6), o.y + (int)((n0 >> 3) & 7u), o.z + (int)(n0 & 7u));
}

// Cells met by voxel coordinate p along one axis: base, base + 1, ... (n of them).
struct AxisCells {
  int base, n;
};
__device__ __forceinline__ AxisCells axis_cells(int p, int o, int S, int h) {
  const int64_t c0 = floor_div((int64_t)p - o, S);
  const int64_t r = (int64_t)p - o - c0 * S;  // 0 <= r < S
  AxisCells a;
  a.base = (int)(c0 - (r < h ? 1 : 0));
  a.n = 1 + (r < h ? 1 : 0) + (r >= S - h ? 1 : 0);
  return a;
}

// Tent of cell c along one axis at the centre of the item at p (p in the widened
// box): twice the distance to the lower face is a = 2 (p - (o + cS - h)) + half2,
// half2 = 1 for a voxel (centre p + 1/2), 8 for a leaf slot (centre p + 4).
__device__ __forceinline__ float tent(int p, int c, int o, int S, int h, int half2) {
  const int64_t a = 2 * ((int64_t)p - ((int64_t)o + (int64_t)c * S - h)) + half2;
  const int m = (int)min(min(a, (int64_t)2 * (S + 2 * h) - a), (int64_t)4 * h);
  return (float)m / (float)(4 * h);
}

__device__ __forceinline__ int expert_at(const MoeGrid& g, const int32_t* __restrict__ table, int cx, int cy, int cz) {
  const int ix = cx - g.clo[0], iy = cy - g.clo[1], iz = cz - g.clo[2];
  if ((unsigned)ix >= (unsigned)g.cdim[0] || (unsigned)iy >= (unsigned)g.cdim[1] || (unsigned)iz >= (unsigned)g.cdim[2])
    return -1;
  return table[((int64_t)ix * g.cdim[1] + iy) * g.cdim[2] + iz];
}

// Calls f(slot j, expert k, gate) for every expert whose widened box holds p,
// in the fixed order j = (ix << 2) | (iy << 1) | iz.
template <class F>
__device__ __forceinline__ void for_each_expert(const MoeGrid& g, const int32_t* __restrict__ table, int3 p, int half2,
                                                F&& f) {
  const AxisCells ax = axis_cells(p.x, g.o[0], g.S, g.h);
  const AxisCells ay = axis_cells(p.y, g.o[1], g.S, g.h);
  const AxisCells az = axis_cells(p.z, g.o[2], g.S, g.h);
  for (int ix = 0; ix < ax.n; ++ix)
    for (int iy = 0; iy < ay.n; ++iy)
      for (int iz = 0; iz < az.n; ++iz) {
        const int cx = ax.base + ix, cy = ay.base + iy, cz = az.base + iz;
        const int k = expert_at(g, table, cx, cy, cz);
        if (k < 0) continue;
        const float w = tent(p.x, cx, g.o[0], g.S, g.h, half2) * tent(p.y, cy, g.o[1], g.S, g.h, half2) *
                        tent(p.z, cz, g.o[2], g.S, g.h, half2);
        f((ix << 2) | (iy << 1) | iz, k, w);
      }
}

// Expert of slot j (j = (ix << 2) | (iy << 1) | iz) for a voxel whose candidate
// cells are ax, ay, az, or -1.
__device__ __forceinline__ int slot_expert(const MoeGrid& g, const int32_t* __restrict__ table, const AxisCells& ax,
                                           const AxisCells& ay, const AxisCells& az, int j) {
  const int ix = j >> 2, iy = (j >> 1) & 1, iz = j & 1;
  if (ix >= ax.n || iy >= ay.n || iz >= az.n) return -1;
  return expert_at(g, table, ax.base + ix, ay.base + iy, az.base + iz);
}

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = (int)(threadIdx.x & 63u);
  return (1ull << lane) - 1ull;
}

// Adds one per lane with k >= 0 to hist[k], one LDS atomic per distinct k in
// the wave; returns each lane's position among the adds to its bin.  Every lane
// of the wave must call it (the loop runs on wave-uniform ballots).
__device__ __forceinline__ uint32_t wave_hist_add(uint32_t* hist, int k) {
  uint32_t pos = 0;
  uint64_t pending = __ballot(k >= 0);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int kl = __shfl(k, leader);
    const uint64_t m = __ballot(k == kl);
    uint32_t base = 0;
    if ((int)(threadIdx.x & 63u) == leader) base = atomicAdd(&hist[kl], (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    if (k == kl) pos = base + (uint32_t)__popcll(m & lanes_below());
    pending &= ~m;
  }
  return pos;
}

// Bounding box of the leaf origins (init: INT_MAX x3, INT_MIN x3).
__global__ void __launch_bounds__(256) k_leaf_bbox(const int4* __restrict__ leaf_o, int64_t n, int* __restrict__ box) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN};
  if (l < n) {
    const int4 o = leaf_o[l];
    mn[0] = mx[0] = o.x;
    mn[1] = mx[1] = o.y;
    mn[2] = mx[2] = o.z;
  }
  for (int d = 0; d < 3; ++d)
    for (int s = 32; s >= 1; s >>= 1) {
      mn[d] = min(mn[d], __shfl_xor(mn[d], s));
      mx[d] = max(mx[d], __shfl_xor(mx[d], s));
    }
  if ((threadIdx.x & 63) == 0) {
    for (int d = 0; d < 3; ++d) {
      atomicMin(&box[d], mn[d]);
      atomicMax(&box[3 + d], mx[d]);
    }
  }
}

// Flags the core cell of every voxel (cells outside the range are ignored; the
// host sizes the range to hold them all).
__global__ void __launch_bounds__(256) k_moe_mark(const int4* __restrict__ leaf_o, const uint32_t* __restrict__ key,
                                                  int64_t n, MoeGrid g, uint8_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int3 p = voxel_of(leaf_o, key[i]);
  const int64_t ix = floor_div((int64_t)p.x - g.o[0], g.S) - g.clo[0];
  const int64_t iy = floor_div((int64_t)p.y - g.o[1], g.S) - g.clo[1];
  const int64_t iz = floor_div((int64_t)p.z - g.o[2], g.S) - g.clo[2];
  if (ix >= 0 && ix < g.cdim[0] && iy >= 0 && iy < g.cdim[1] && iz >= 0 && iz < g.cdim[2])
    flag[(ix * g.cdim[1] + iy) * g.cdim[2] + iz] = 1;
}

// Per active tile: every cell whose core meets the tile's 8^3 region (a tile
// straddles several cores when the grid is not aligned to 8).
__global__ void __launch_bounds__(256) k_moe_mark_tiles(const int4* __restrict__ l1_o,
                                                        const uint32_t* __restrict__ tkey, int64_t n, MoeGrid g,
                                                        uint8_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = tkey[i], n1 = k & 4095u;
  const int4 o = l1_o[k >> 12];
  const int p[3] = {o.x + 8 * (int)(n1 >> 8), o.y + 8 * (int)((n1 >> 4) & 15u), o.z + 8 * (int)(n1 & 15u)};
  int64_t a[3], b[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    a[d] = max(floor_div((int64_t)p[d] - g.o[d], g.S) - g.clo[d], (int64_t)0);
    b[d] = min(floor_div((int64_t)p[d] + 7 - g.o[d], g.S) - g.clo[d], (int64_t)g.cdim[d] - 1);
  }
  for (int64_t ix = a[0]; ix <= b[0]; ++ix)
    for (int64_t iy = a[1]; iy <= b[1]; ++iy)
      for (int64_t iz = a[2]; iz <= b[2]; ++iz) flag[(ix * g.cdim[1] + iy) * g.cdim[2] + iz] = 1;
}

// Voxels inside a widened box [lo, lo + D)^3, appended (one global atomic per
// block): with `tiles` false item i is voxel i (origins leaf_o, keys key, values
// val); with `tiles` true it is voxel i & 511 of active tile i >> 9 (level-1
// origins leaf_o, tile keys key, tile values val), every voxel of a tile holding
// the tile's value.
__global__ void __launch_bounds__(256) k_moe_extract(const int4* __restrict__ leaf_o, const uint32_t* __restrict__ key,
                                                     const float* __restrict__ val, int64_t n, bool tiles, int lx,
                                                     int ly, int lz, int D, int32_t* __restrict__ ijk,
                                                     float* __restrict__ v, uint32_t* __restrict__ count) {
  __shared__ uint32_t wcount[4], wbase[4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int w = (int)(threadIdx.x >> 6);
  bool in = false;
  int3 p = make_int3(0, 0, 0);
  if (i < n) {
    if (tiles) {
      const uint32_t k = key[i >> 9], n1 = k & 4095u, n0 = (uint32_t)(i & 511);
      const int4 o = leaf_o[k >> 12];
      p = make_int3(o.x + 8 * (int)(n1 >> 8) + (int)(n0 >> 6), o.y + 8 * (int)((n1 >> 4) & 15u) + (int)((n0 >> 3) & 7u),
                    o.z + 8 * (int)(n1 & 15u) + (int)(n0 & 7u));
    } else {
      p = voxel_of(leaf_o, key[i]);
    }
    in = (int64_t)p.x - lx >= 0 && (int64_t)p.x - lx < D && (int64_t)p.y - ly >= 0 && (int64_t)p.y - ly < D &&
         (int64_t)p.z - lz >= 0 && (int64_t)p.z - lz < D;
  }
  const uint64_t b = __ballot(in);
  if ((threadIdx.x & 63u) == 0) wcount[w] = (uint32_t)__popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t t = wcount[0] + wcount[1] + wcount[2] + wcount[3];
    uint32_t s = t ? atomicAdd(count, t) : 0u;
    for (int k = 0; k < 4; ++k) {
      wbase[k] = s;
      s += wcount[k];
    }
  }
  __syncthreads();
  if (in) {
    const uint32_t s = wbase[w] + (uint32_t)__popcll(b & lanes_below());
    ijk[3 * (size_t)s] = p.x;
    ijk[3 * (size_t)s + 1] = p.y;
    ijk[3 * (size_t)s + 2] = p.z;
    v[s] = val[tiles ? i >> 9 : i];
  }
}

// Item i is voxel i (key[i] = leaf << 9 | n0), or, with key null, voxel slot i of
// the leaves (i = leaf << 9 | n0 itself), or (l1) leaf slot k & 4095 of level-1
// node k >> 12, positioned at the slot's origin, with k = i, or k = key[i] for the
// active tiles.
__device__ __forceinline__ int3 item_of(const ItemSrc& s, int64_t i) {
  if (s.l1) {
    const int64_t k = s.key ? (int64_t)s.key[i] : i;
    const int4 o = s.org[k >> 12];
    const int n1 = (int)(k & 4095);
    return make_int3(o.x + 8 * (n1 >> 8), o.y + 8 * ((n1 >> 4) & 15), o.z + 8 * (n1 & 15));
  }
  return voxel_of(s.org, s.key ? s.key[i] : (uint32_t)i);
}

// Candidate cells of item i (none past n).
__device__ __forceinline__ void voxel_cells(const ItemSrc& src, int64_t i, int64_t n, const MoeGrid& g, int3& p,
                                            AxisCells& ax, AxisCells& ay, AxisCells& az) {
  p = make_int3(0, 0, 0);
  ax = ay = az = AxisCells{0, 0};
  if (i < n) {
    p = item_of(src, i);
    ax = axis_cells(p.x, g.o[0], g.S, g.h);
    ay = axis_cells(p.y, g.o[1], g.S, g.h);
    az = axis_cells(p.z, g.o[2], g.S, g.h);
  }
}

// Pass 1 of the routing: (voxel, expert) pairs per expert, and voxels no expert
// covers.  Each block walks several 256-voxel tiles (block-uniform trip count)
// into an LDS histogram (wave-aggregated adds), then adds it to the global
// counts with one atomic per (block, expert).
__global__ void __launch_bounds__(256) k_moe_count(ItemSrc src, int64_t n, MoeGrid g, const int32_t* __restrict__ table,
                                                   int n_exp, uint32_t* __restrict__ cnt,
                                                   uint32_t* __restrict__ uncovered) {
  extern __shared__ uint32_t lds[];  // n_exp counters, sized at launch
  uint32_t* hist = lds;
  __shared__ uint32_t unc;
  for (int k = threadIdx.x; k < n_exp; k += blockDim.x) hist[k] = 0u;
  if (threadIdx.x == 0) unc = 0u;
  __syncthreads();
  for (int64_t t0 = (int64_t)blockIdx.x * 256; t0 < n; t0 += (int64_t)gridDim.x * 256) {
    const int64_t i = t0 + threadIdx.x;
    int3 p;
    AxisCells ax, ay, az;
    voxel_cells(src, i, n, g, p, ax, ay, az);
    bool covered = false;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = slot_expert(g, table, ax, ay, az, j);
      covered |= k >= 0;
      (void)wave_hist_add(hist, k);
    }
    const uint64_t bad = __ballot(i < n && !covered);
    if ((threadIdx.x & 63u) == 0 && bad) atomicAdd(&unc, (uint32_t)__popcll(bad));
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n_exp; k += blockDim.x)
    if (hist[k]) atomicAdd(&cnt[k], hist[k]);
  if (threadIdx.x == 0 && unc) atomicAdd(uncovered, unc);
}

// Pass 2: writes each pair into its expert's bucket: the expert's normalised
// coordinates and the item's slot j n + i.  A block counts its pairs per
// expert, reserves one range per expert after `start[k]` with one atomic, then
// walks its tiles again and fills the ranges (positions from fresh LDS
// counters: any order within a range will do).
__global__ void __launch_bounds__(256) k_moe_route(ItemSrc src, int64_t n, MoeGrid g, const int32_t* __restrict__ table,
                                                   const MoeBox* __restrict__ box, int n_exp,
                                                   const uint32_t* __restrict__ start, uint32_t* __restrict__ cursor,
                                                   float* __restrict__ bx, uint32_t* __restrict__ bslot, uint64_t cap) {
  extern __shared__ uint32_t lds[];  // 3 n_exp words, sized at launch
  uint32_t* hist = lds;
  uint32_t* base = lds + n_exp;
  uint32_t* fill = lds + 2 * n_exp;
  for (int k = threadIdx.x; k < n_exp; k += blockDim.x) hist[k] = fill[k] = 0u;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t t0 = (int64_t)blockIdx.x * 256; t0 < n; t0 += stride) {
    int3 p;
    AxisCells ax, ay, az;
    voxel_cells(src, t0 + threadIdx.x, n, g, p, ax, ay, az);
#pragma unroll
    for (int j = 0; j < 8; ++j) (void)wave_hist_add(hist, slot_expert(g, table, ax, ay, az, j));
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n_exp; k += blockDim.x) base[k] = hist[k] ? start[k] + atomicAdd(&cursor[k], hist[k]) : 0u;
  __syncthreads();
  for (int64_t t0 = (int64_t)blockIdx.x * 256; t0 < n; t0 += stride) {
    const int64_t i = t0 + threadIdx.x;
    int3 p;
    AxisCells ax, ay, az;
    voxel_cells(src, i, n, g, p, ax, ay, az);
    const float half = src.l1 ? 4.f : 0.5f;  // the item's centre
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = slot_expert(g, table, ax, ay, az, j);
      const uint32_t pos = wave_hist_add(fill, k);
      if (k < 0) continue;
      const uint32_t s = base[k] + pos;
      if (s >= cap) continue;  // the pair buffers were too small: the caller retries
      const MoeBox b = box[k];
      bx[3 * (size_t)s] = ((float)(p.x - b.lo[0]) + half) * b.inv_d;
      bx[3 * (size_t)s + 1] = ((float)(p.y - b.lo[1]) + half) * b.inv_d;
      bx[3 * (size_t)s + 2] = ((float)(p.z - b.lo[2]) + half) * b.inv_d;
      bslot[s] = (uint32_t)j * (uint32_t)n + (uint32_t)i;
    }
  }
}

// The same two passes for voxel and voxel-slot items when the cell grid is
// leaf-aligned (origin, edge and halo multiples of 8): every item of a leaf then
// meets the same experts, so the experts are found once per leaf and its m items
// (its active voxels, or its 512 slots) are counted and reserved together.
__device__ __forceinline__ void leaf_cells(const int4& o, const MoeGrid& g, AxisCells& ax, AxisCells& ay,
                                           AxisCells& az) {
  ax = axis_cells(o.x, g.o[0], g.S, g.h);
  ay = axis_cells(o.y, g.o[1], g.S, g.h);
  az = axis_cells(o.z, g.o[2], g.S, g.h);
}
__device__ __forceinline__ uint32_t leaf_items(const uint32_t* __restrict__ leaf_off, int64_t l) {
  return leaf_off ? leaf_off[l + 1] - leaf_off[l] : 512u;
}

__global__ void __launch_bounds__(256) k_moe_count_leaf(const int4* __restrict__ leaf_o,
                                                        const uint32_t* __restrict__ leaf_off, int64_t n_leaf,
                                                        MoeGrid g, const int32_t* __restrict__ table, int n_exp,
                                                        uint32_t* __restrict__ cnt, uint32_t* __restrict__ uncovered) {
  extern __shared__ uint32_t lds[];  // n_exp counters
  __shared__ uint32_t unc;
  for (int k = threadIdx.x; k < n_exp; k += blockDim.x) lds[k] = 0u;
  if (threadIdx.x == 0) unc = 0u;
  __syncthreads();
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n_leaf; l += (int64_t)gridDim.x * blockDim.x) {
    AxisCells ax, ay, az;
    leaf_cells(leaf_o[l], g, ax, ay, az);
    const uint32_t m = leaf_items(leaf_off, l);
    bool covered = false;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = slot_expert(g, table, ax, ay, az, j);
      if (k >= 0) {
        atomicAdd(&lds[k], m);
        covered = true;
      }
    }
    if (!covered && m) atomicAdd(&unc, m);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n_exp; k += blockDim.x)
    if (lds[k]) atomicAdd(&cnt[k], lds[k]);
  if (threadIdx.x == 0 && unc) atomicAdd(uncovered, unc);
}

// One wave per leaf: walk 1 sums the block's items per expert, one global atomic
// per (block, expert) reserves its ranges, walk 2 gives each (leaf, expert) a run
// of m consecutive places in the range and the lanes fill it.
__global__ void __launch_bounds__(256) k_moe_route_leaf(const int4* __restrict__ leaf_o,
                                                        const uint32_t* __restrict__ leaf_off,
                                                        const uint32_t* __restrict__ key, int64_t n_leaf, MoeGrid g,
                                                        const int32_t* __restrict__ table,
                                                        const MoeBox* __restrict__ box, int n_exp,
                                                        const uint32_t* __restrict__ start,
                                                        uint32_t* __restrict__ cursor, float* __restrict__ bx,
                                                        uint32_t* __restrict__ bslot, uint32_t n_items,
                                                        uint64_t cap) {
  extern __shared__ uint32_t lds[];  // 3 n_exp words
  uint32_t* hist = lds;
  uint32_t* base = lds + n_exp;
  uint32_t* fill = lds + 2 * n_exp;
  for (int k = threadIdx.x; k < n_exp; k += blockDim.x) hist[k] = fill[k] = 0u;
  __syncthreads();
  const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63u);
  const int64_t stride = (int64_t)gridDim.x * 4;
  for (int64_t l = (int64_t)blockIdx.x * 4 + wave; l < n_leaf; l += stride) {
    if (lane != 0) continue;
    AxisCells ax, ay, az;
    leaf_cells(leaf_o[l], g, ax, ay, az);
    const uint32_t m = leaf_items(leaf_off, l);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = slot_expert(g, table, ax, ay, az, j);
      if (k >= 0 && m) atomicAdd(&hist[k], m);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n_exp; k += blockDim.x) base[k] = hist[k] ? start[k] + atomicAdd(&cursor[k], hist[k]) : 0u;
  __syncthreads();
  for (int64_t l = (int64_t)blockIdx.x * 4 + wave; l < n_leaf; l += stride) {
    const int4 o = leaf_o[l];
    AxisCells ax, ay, az;
    leaf_cells(o, g, ax, ay, az);
    const uint32_t m = leaf_items(leaf_off, l);
    const uint32_t i0 = leaf_off ? leaf_off[l] : (uint32_t)(l * 512);
#pragma unroll 1
    for (int j = 0; j < 8; ++j) {
      const int k = slot_expert(g, table, ax, ay, az, j);  // wave-uniform
      if (k < 0 || m == 0) continue;
      uint32_t run = 0;
      if (lane == 0) run = atomicAdd(&fill[k], m);
      run = __shfl(run, 0);
      const MoeBox b = box[k];
      for (uint32_t r = lane; r < m; r += 64) {
        const uint32_t i = i0 + r;
        const uint32_t n0 = key ? (key[i] & 511u) : r;
        const uint64_t s = (uint64_t)base[k] + run + r;
        if (s >= cap) continue;  // the pair buffers were too small: the caller retries
        const int px = o.x + (int)(n0 >> 6), py = o.y + (int)((n0 >> 3) & 7u), pz = o.z + (int)(n0 & 7u);
        bx[3 * s] = ((float)(px - b.lo[0]) + 0.5f) * b.inv_d;
        bx[3 * s + 1] = ((float)(py - b.lo[1]) + 0.5f) * b.inv_d;
        bx[3 * s + 2] = ((float)(pz - b.lo[2]) + 0.5f) * b.inv_d;
        bslot[s] = (uint32_t)j * n_items + i;
      }
    }
  }
}

// Gate-weighted average of the expert outputs held in the item's 8 slots: a
// value per voxel (or per active tile, gated at the tile's centre), or (mask
// non-null) the bit "blended logit > 0" per voxel slot, packed 64 to a word by the
// wave that computed them, or (cls non-null, leaf-slot items) the class of the
// three blended logits (argmax, ties to the lowest).
__global__ void __launch_bounds__(256) k_moe_blend(ItemSrc src, int64_t n, MoeGrid g,
                                                   const int32_t* __restrict__ table,
                                                   const float* __restrict__ yslot, float* __restrict__ values,
                                                   uint64_t* __restrict__ mask, uint8_t* __restrict__ cls) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float v = 0.f;
  if (i < n && cls) {
    const int3 p = item_of(src, i);
    float num[3] = {0.f, 0.f, 0.f}, den = 0.f;
    for_each_expert(g, table, p, 8, [&](int j, int, float w) {
#pragma unroll
      for (int c = 0; c < 3; ++c) num[c] += w * yslot[3 * ((size_t)j * n + i) + c];
      den += w;
    });
    int best = 0;
#pragma unroll
    for (int c = 1; c < 3; ++c)
      if (num[c] / den > num[best] / den) best = c;
    cls[i] = den > 0.f ? (uint8_t)best : (uint8_t)255;
    return;
  }
  if (i < n) {
    const int3 p = item_of(src, i);
    float num = 0.f, den = 0.f;
    for_each_expert(g, table, p, src.l1 ? 8 : 1, [&](int j, int, float w) {
      num += w * yslot[(size_t)j * n + i];
      den += w;
    });
    v = den > 0.f ? num / den : __builtin_nanf("");
    if (values) values[i] = v;
  }
  if (mask) {
    const uint64_t bits = __ballot(i < n && v > 0.f);
    if ((threadIdx.x & 63u) == 0 && i < n) mask[i >> 6] = bits;
  }
}

// The mask blend per leaf of a leaf-aligned grid: one wave per leaf, whose 512
// voxel slots i = 512 l + r all lie in the same widened boxes, so the leaf's
// experts are looked up once; each lane blends slots r = lane, lane + 64, ... with
// k_moe_blend's order and arithmetic (j ascending, gate = product of the three
// tents at the voxel centre) and the wave packs each 64 bits into a mask word.
// (For the voxels of a level set, about 180 per leaf, one thread per voxel is
// faster: the wave's passes over a leaf would chain their loads.)
__global__ void __launch_bounds__(256) k_moe_blend_slots_leaf(const int4* __restrict__ leaf_o, int64_t n_leaf,
                                                              MoeGrid g, const int32_t* __restrict__ table,
                                                              const float* __restrict__ yslot,
                                                              uint64_t* __restrict__ mask) {
  const int64_t l = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  if (l >= n_leaf) return;  // uniform per wave
  const size_t n = 512 * (size_t)n_leaf;
  const int4 o = leaf_o[l];
  AxisCells ax, ay, az;
  leaf_cells(o, g, ax, ay, az);
  int kj[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) kj[j] = slot_expert(g, table, ax, ay, az, j);
#pragma unroll 1
  for (uint32_t r0 = 0; r0 < 512; r0 += 64) {
    const uint32_t r = r0 + lane;
    const size_t i = 512 * (size_t)l + r;
    const int px = o.x + (int)(r >> 6), py = o.y + (int)((r >> 3) & 7u), pz = o.z + (int)(r & 7u);
    float num = 0.f, den = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (kj[j] < 0) continue;
      const float w = tent(px, ax.base + (j >> 2), g.o[0], g.S, g.h, 1) *
                      tent(py, ay.base + ((j >> 1) & 1), g.o[1], g.S, g.h, 1) *
                      tent(pz, az.base + (j & 1), g.o[2], g.S, g.h, 1);
      num += w * yslot[(size_t)j * n + i];
      den += w;
    }
    const float v = den > 0.f ? num / den : __builtin_nanf("");
    const uint64_t bits = __ballot(v > 0.f);
    if (lane == 0) mask[(size_t)l * 8 + (r0 >> 6)] = bits;
  }
}

unsigned grid_of(int64_t n) { return (unsigned)((n + 255) / 256); }
// the routing passes: at most four blocks per compute unit, each walking several tiles
unsigned route_grid(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 1024); }

}  // namespace

void leaf_bbox(const Tree& t, int32_t lo[3], int32_t hi[3], hipStream_t st) {
  const int init[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN};
  DevBuf<int> box;
  box.alloc(6);
  NVDB_HIP(hipMemcpyAsync(box.p, init, sizeof(init), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_leaf_bbox, dim3(grid_of(t.n_leaf)), dim3(256), 0, st, t.leaf_o.p, t.n_leaf, box.p);
  NVDB_HIP(hipGetLastError());
  int h[6];
  NVDB_HIP(hipMemcpyAsync(h, box.p, sizeof(h), hipMemcpyDeviceToHost, st));
  NVDB_HIP(hipStreamSynchronize(st));
  for (int d = 0; d < 3; ++d) {
    lo[d] = h[d];
    hi[d] = h[3 + d] + 8;  // leaves span 8 voxels
  }
}

void moe_mark_cells(const Tree& t, const MoeGrid& g, uint8_t* flag, hipStream_t st) {
  if (t.n_vox > 0) {
    hipLaunchKernelGGL(k_moe_mark, dim3(grid_of(t.n_vox)), dim3(256), 0, st, t.leaf_o.p, t.vox_key.p, t.n_vox, g,
                       flag);
    NVDB_HIP(hipGetLastError());
  }
  if (t.n_tile > 0) {
    hipLaunchKernelGGL(k_moe_mark_tiles, dim3(grid_of(t.n_tile)), dim3(256), 0, st, t.l1_o.p, t.tile_key.p, t.n_tile,
                       g, flag);
    NVDB_HIP(hipGetLastError());
  }
}

int64_t moe_extract(const Tree& t, const int32_t lo[3], int32_t D, int32_t* ijk, float* v, uint32_t* count,
                    hipStream_t st) {
  NVDB_HIP(hipMemsetAsync(count, 0, sizeof(uint32_t), st));
  if (t.n_vox > 0) {
    hipLaunchKernelGGL(k_moe_extract, dim3(grid_of(t.n_vox)), dim3(256), 0, st, t.leaf_o.p, t.vox_key.p, t.values.p,
                       t.n_vox, false, lo[0], lo[1], lo[2], D, ijk, v, count);
    NVDB_HIP(hipGetLastError());
  }
  if (t.n_tile > 0) {  // the voxels of the active tiles, appended after the others
    hipLaunchKernelGGL(k_moe_extract, dim3(grid_of(512 * t.n_tile)), dim3(256), 0, st, t.l1_o.p, t.tile_key.p,
                       t.tile_val.p, 512 * t.n_tile, true, lo[0], lo[1], lo[2], D, ijk, v, count);
    NVDB_HIP(hipGetLastError());
  }
  uint32_t c = 0;
  NVDB_HIP(hipMemcpyAsync(&c, count, sizeof(c), hipMemcpyDeviceToHost, st));
  NVDB_HIP(hipStreamSynchronize(st));
  return (int64_t)c;
}

static int64_t items(const Tree& t, int kind) {
  if (kind == MOE_TILES) return t.n_tile;
  return kind == MOE_VOXELS ? t.n_vox : (kind == MOE_VOXEL_SLOTS ? 512 * t.n_leaf : 4096 * t.n_l1);
}
static ItemSrc item_src(const Tree& t, int kind) {
  if (kind == MOE_LEAF_SLOTS) return ItemSrc{t.l1_o.p, nullptr, 1};
  if (kind == MOE_TILES) return ItemSrc{t.l1_o.p, t.tile_key.p, 1};
  return ItemSrc{t.leaf_o.p, kind == MOE_VOXELS ? t.vox_key.p : nullptr, 0};
}

// Voxel and voxel-slot items of a leaf-aligned grid are routed per leaf.
static bool per_leaf(const MoeGrid& g, int kind) {
  return (kind == MOE_VOXELS || kind == MOE_VOXEL_SLOTS) && ((g.o[0] | g.o[1] | g.o[2] | g.S | g.h) & 7) == 0;
}
static unsigned leaf_grid(int64_t n_leaf, int per_block, int64_t max_blocks) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(max_blocks, (n_leaf + per_block - 1) / per_block));
}

void moe_count(const Tree& t, int kind, const MoeGrid& g, const int32_t* table, int n_exp, uint32_t* cnt,
               uint32_t* uncovered, hipStream_t st) {
  if (per_leaf(g, kind)) {
    if (t.n_leaf == 0) return;
    hipLaunchKernelGGL(k_moe_count_leaf, dim3(leaf_grid(t.n_leaf, 256, 1024)), dim3(256), (size_t)n_exp * 4, st, t.leaf_o.p,
                       kind == MOE_VOXELS ? t.leaf_off.p : nullptr, t.n_leaf, g, table, n_exp, cnt, uncovered);
  } else {
    hipLaunchKernelGGL(k_moe_count, dim3(route_grid(items(t, kind))), dim3(256), (size_t)n_exp * 4, st,
                       item_src(t, kind), items(t, kind), g, table, n_exp, cnt, uncovered);
  }
  NVDB_HIP(hipGetLastError());
}

void moe_route(const Tree& t, int kind, const MoeGrid& g, const int32_t* table, const MoeBox* box, int n_exp,
               const uint32_t* start, uint32_t* cursor, float* bx, uint32_t* bslot, uint64_t cap, hipStream_t st) {
  if (per_leaf(g, kind)) {
    if (t.n_leaf == 0) return;
    const bool vox = kind == MOE_VOXELS;
    hipLaunchKernelGGL(k_moe_route_leaf, dim3(leaf_grid(t.n_leaf, 4, 1024)), dim3(256), (size_t)n_exp * 12, st, t.leaf_o.p,
                       vox ? t.leaf_off.p : nullptr, vox ? t.vox_key.p : nullptr, t.n_leaf, g, table, box, n_exp,
                       start, cursor, bx, bslot, (uint32_t)items(t, kind), cap);
  } else {
    hipLaunchKernelGGL(k_moe_route, dim3(route_grid(items(t, kind))), dim3(256), (size_t)n_exp * 12, st,
                       item_src(t, kind), items(t, kind), g, table, box, n_exp, start, cursor, bx, bslot, cap);
  }
  NVDB_HIP(hipGetLastError());
}

namespace {
// One work-group of 256 threads; n <= 4096 experts, each thread a contiguous run.
// When the padded pairs exceed cap, flag[0] is set and the chunk count is 0 (the
// grouped decode then does nothing and the caller retries with larger buffers).
// flag[1] receives cnt[n], the count of items no expert holds, so that one copy
// brings both back.
__global__ void __launch_bounds__(256) k_moe_plan(const uint32_t* __restrict__ cnt, int n, int chunk, uint64_t cap,
                                                  uint32_t* __restrict__ cs, uint32_t* __restrict__ start,
                                                  uint32_t* __restrict__ flag) {
  __shared__ uint32_t part[256];
  const int per = (n + 255) / 256, k0 = threadIdx.x * per, k1 = min(n, k0 + per);
  uint32_t sum = 0;
  for (int k = k0; k < k1; ++k) sum += (cnt[k] + (uint32_t)chunk - 1) / (uint32_t)chunk;
  part[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {  // exclusive scan of the 256 partial sums
    uint32_t run = 0;
    for (int i = 0; i < 256; ++i) {
      const uint32_t v = part[i];
      part[i] = run;
      run += v;
    }
    const bool over = (uint64_t)run * (uint64_t)chunk > cap;
    cs[n] = over ? 0u : run;
    flag[0] = over ? 1u : 0u;
    flag[1] = cnt[n];
  }
  __syncthreads();
  uint32_t run = part[threadIdx.x];
  for (int k = k0; k < k1; ++k) {
    cs[k] = run;
    start[k] = run * (uint32_t)chunk;
    run += (cnt[k] + (uint32_t)chunk - 1) / (uint32_t)chunk;
  }
}
}  // namespace

void moe_plan(const uint32_t* cnt, int n, int chunk, uint64_t cap, uint32_t* cs, uint32_t* start, uint32_t* flag,
              hipStream_t st) {
  hipLaunchKernelGGL(k_moe_plan, dim3(1), dim3(256), 0, st, cnt, n, chunk, cap, cs, start, flag);
  NVDB_HIP(hipGetLastError());
}

void moe_blend(const Tree& t, int kind, const MoeGrid& g, const int32_t* table, const float* yslot, float* values,
               uint64_t* mask, uint8_t* cls, hipStream_t st) {
  if (kind == MOE_VOXEL_SLOTS && per_leaf(g, kind)) {
    if (t.n_leaf == 0) return;
    hipLaunchKernelGGL(k_moe_blend_slots_leaf, dim3((unsigned)((t.n_leaf + 3) / 4)), dim3(256), 0, st, t.leaf_o.p,
                       t.n_leaf, g, table, yslot, mask);
  } else {
    hipLaunchKernelGGL(k_moe_blend, dim3(grid_of(items(t, kind))), dim3(256), 0, st, item_src(t, kind), items(t, kind),
                       g, table, yslot, values, mask, cls);
  }
  NVDB_HIP(hipGetLastError());
}

}  // namespace nvdb
