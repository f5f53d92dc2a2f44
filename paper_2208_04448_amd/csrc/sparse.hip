// VDB [Hash,5,4,3] tree build from a sparse voxel list (NeuralVDB Sec. 3.1).
//
// Every voxel gets a 63-bit key whose ascending order is the canonical order of
// the tree: the level-2 node (x>>12, y>>12, z>>12, each biased into 9 bits),
// then its slot n2 (15 bits), the level-1 slot n1 (12 bits) and the leaf slot
// n0 (9 bits).  A stable LSD radix sort of (key, input position) pairs puts the
// voxels in tree order, and equal neighbours are duplicates.  The active rule
// is applied after the sort (so duplicates are caught whatever their values),
// and flags where the leaf or level-1 part of the key changes, with their
// scans, number the nodes.  The arrays are the ones the dense build produces.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "nvdb_internal.h"

namespace nvdb {

namespace {

constexpr int COORD_LIM = 1 << 20;  // coordinates lie in [-2^20, 2^20)
constexpr int RS_THREADS = 256, RS_ITEMS = 8, RS_TILE = RS_THREADS * RS_ITEMS;
constexpr int RS_BINS = 256, RS_PASSES = 8;  // 8-bit digits over the 64-bit key

enum : int { BAD_VALUE = 1, BAD_RANGE = 2, BAD_DUPLICATE = 4 };

__device__ __forceinline__ uint64_t voxel_key(int x, int y, int z) {
  const uint64_t hx = (uint64_t)((x >> 12) + 256), hy = (uint64_t)((y >> 12) + 256), hz = (uint64_t)((z >> 12) + 256);
  const uint64_t n2 = (uint64_t)((((x >> 7) & 31) << 10) | (((y >> 7) & 31) << 5) | ((z >> 7) & 31));
  const uint64_t n1 = (uint64_t)((((x >> 3) & 15) << 8) | (((y >> 3) & 15) << 4) | ((z >> 3) & 15));
  const uint64_t n0 = (uint64_t)(((x & 7) << 6) | ((y & 7) << 3) | (z & 7));
  return (hx << 54) | (hy << 45) | (hz << 36) | (n2 << 21) | (n1 << 9) | n0;
}

// Coordinate d (0 = x, 1 = y, 2 = z) of the voxel with key k.
__device__ __forceinline__ int key_coord(uint64_t k, int d) {
  const int hi = (int)((k >> (54 - 9 * d)) & 511) - 256;
  const int s2 = (int)((k >> (21 + 10 - 5 * d)) & 31);
  const int s1 = (int)((k >> (9 + 8 - 4 * d)) & 15);
  const int s0 = (int)((k >> (6 - 3 * d)) & 7);
  return hi * 4096 + (s2 << 7) + (s1 << 3) + s0;
}

__device__ __forceinline__ bool is_active(int kind, float thr, float v) {
  return kind == NVDB_SDF ? (fabsf(v) <= thr) : (v > thr);
}

// Keys, input positions, value / range checks and the bounding box
// (bbox[0..2] minima, bbox[3..5] maxima).
__global__ void __launch_bounds__(256) k_sp_keys(const int32_t* __restrict__ ijk, const float* __restrict__ v, int64_t n,
                                                 uint64_t* __restrict__ key, uint32_t* __restrict__ pos, int* bad,
                                                 int* bbox) {
  int mn[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, mx[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
  int flags = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int x = ijk[3 * i], y = ijk[3 * i + 1], z = ijk[3 * i + 2];
    const float f = v[i];
    if (!isfinite(f)) flags |= BAD_VALUE;
    const bool in = x >= -COORD_LIM && x < COORD_LIM && y >= -COORD_LIM && y < COORD_LIM && z >= -COORD_LIM &&
                    z < COORD_LIM;
    if (!in) flags |= BAD_RANGE;
    key[i] = in ? voxel_key(x, y, z) : 0;
    pos[i] = (uint32_t)i;
    mn[0] = min(mn[0], x), mn[1] = min(mn[1], y), mn[2] = min(mn[2], z);
    mx[0] = max(mx[0], x), mx[1] = max(mx[1], y), mx[2] = max(mx[2], z);
  }
  // wave reduction, one atomic per wave and quantity
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    flags |= __shfl_xor(flags, off);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      mn[d] = min(mn[d], __shfl_xor(mn[d], off));
      mx[d] = max(mx[d], __shfl_xor(mx[d], off));
    }
  }
  if ((threadIdx.x & 63) == 0) {
    if (flags) atomicOr(bad, flags);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      atomicMin(&bbox[d], mn[d]);
      atomicMax(&bbox[3 + d], mx[d]);
    }
  }
}

// Radix-sort pass, part 1: per-tile digit counts, stored digit-major
// (hist[digit * n_tiles + tile]) so that one exclusive scan gives every
// (digit, tile) pair its output offset.
__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const uint64_t* __restrict__ key, int64_t n, int shift,
                                                        int64_t n_tiles, uint64_t* __restrict__ hist) {
  __shared__ uint32_t h[RS_BINS];
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
  for (int k = 0; k < RS_ITEMS; ++k) {
    const int64_t i = base + k * RS_THREADS + t;
    if (i < n) atomicAdd(&h[(key[i] >> shift) & (RS_BINS - 1)], 1u);
  }
  __syncthreads();
  hist[(int64_t)t * n_tiles + blockIdx.x] = h[t];
}

// Radix-sort pass, part 2: stable scatter.  Elements of a tile are taken in
// input order, RS_THREADS at a time; inside a wave the lanes holding the same
// digit find each other with 8 ballots (one per digit bit), and per-wave digit
// counts in LDS give each wave its base, so ranks follow the input order.
__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const uint64_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin, int64_t n, int shift,
                                                           int64_t n_tiles, const uint64_t* __restrict__ off,
                                                           uint64_t* __restrict__ kout, uint32_t* __restrict__ vout) {
  __shared__ uint32_t wcnt[RS_THREADS / 64][RS_BINS];
  __shared__ uint32_t wbase[RS_THREADS / 64][RS_BINS];
  __shared__ uint32_t run[RS_BINS];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  run[t] = 0;
#pragma unroll
  for (int q = 0; q < RS_THREADS / 64; ++q) wcnt[q][t] = 0;
  const uint64_t tile_off = off[(int64_t)t * n_tiles + blockIdx.x];  // this thread's digit t
  __shared__ uint64_t toff[RS_BINS];
  toff[t] = tile_off;
  __syncthreads();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int k = 0; k < RS_ITEMS; ++k) {
    const int64_t i = base + k * RS_THREADS + t;
    const bool valid = i < n;
    const uint64_t kk = valid ? kin[i] : 0ull;
    const uint32_t vv = valid ? vin[i] : 0u;
    const int d = (int)((kk >> shift) & (RS_BINS - 1));
    uint64_t match = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bal = __ballot(valid && bit);
      match &= bit ? bal : ~bal;
    }
    const int rank = __popcll(match & below);
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(match);
    __syncthreads();
    {
      uint32_t r = run[t];
#pragma unroll
      for (int q = 0; q < RS_THREADS / 64; ++q) {
        wbase[q][t] = r;
        r += wcnt[q][t];
        wcnt[q][t] = 0;
      }
      run[t] = r;
    }
    __syncthreads();
    if (valid) {
      const uint64_t dst = toff[d] + wbase[w][d] + (uint32_t)rank;
      kout[dst] = kk;
      vout[dst] = vv;
    }
  }
}

// Duplicate check on the sorted keys and the active flag of every voxel.
__global__ void __launch_bounds__(256) k_sp_mark(const uint64_t* __restrict__ key, const uint32_t* __restrict__ pos,
                                                 const float* __restrict__ v, int64_t n, int kind, float thr,
                                                 uint64_t* __restrict__ act, int* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (i > 0 && key[i] == key[i - 1]) atomicOr(bad, BAD_DUPLICATE);
    act[i] = is_active(kind, thr, v[pos[i]]) ? 1ull : 0ull;
  }
}

// Active voxels in tree order: keys and values.
__global__ void __launch_bounds__(256) k_sp_compact(const uint64_t* __restrict__ key, const uint32_t* __restrict__ pos,
                                                    const float* __restrict__ v, const uint64_t* __restrict__ act,
                                                    const uint64_t* __restrict__ pre, int64_t n,
                                                    uint64_t* __restrict__ ckey, float* __restrict__ cval) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (act[i]) {
      ckey[pre[i]] = key[i];
      cval[pre[i]] = v[pos[i]];
    }
}

// flag[i] = 1 where key >> shift differs from the previous element's.
__global__ void __launch_bounds__(256) k_sp_starts(const uint64_t* __restrict__ key, int64_t n, int shift,
                                                   uint64_t* __restrict__ flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    flag[i] = (i == 0 || (key[i] >> shift) != (key[i - 1] >> shift)) ? 1ull : 0ull;
}

// Leaves: origin, mask, voxel offset; voxels: value and (leaf << 9 | n0).
__global__ void __launch_bounds__(256) k_sp_leaves(const uint64_t* __restrict__ ckey, const float* __restrict__ cval,
                                                   int64_t n, const uint64_t* __restrict__ flag,
                                                   const uint64_t* __restrict__ pre, int4* __restrict__ leaf_o,
                                                   uint64_t* leaf_mask, uint32_t* __restrict__ leaf_off,
                                                   float* __restrict__ values, uint32_t* __restrict__ vox_key,
                                                   uint64_t* __restrict__ leaf_key) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = ckey[j];
    const int64_t leaf = (int64_t)(pre[j] + flag[j]) - 1;
    const uint32_t n0 = (uint32_t)(k & 511);
    values[j] = cval[j];
    vox_key[j] = ((uint32_t)leaf << 9) | n0;
    if (flag[j]) {
      leaf_off[leaf] = (uint32_t)j;
      leaf_o[leaf] = make_int4(key_coord(k, 0) & ~7, key_coord(k, 1) & ~7, key_coord(k, 2) & ~7, 0);
      leaf_key[leaf] = k >> 9;
    }
    atomicOr((unsigned long long*)&leaf_mask[leaf * 8 + (n0 >> 6)], 1ull << (n0 & 63));
  }
}

// Level-1 nodes: origin and child mask (bit n1 for every leaf).
__global__ void __launch_bounds__(256) k_sp_l1(const uint64_t* __restrict__ leaf_key, int64_t n_leaf,
                                               const uint64_t* __restrict__ flag, const uint64_t* __restrict__ pre,
                                               int4* __restrict__ l1_o, uint64_t* l1_child) {
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < n_leaf; l += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = leaf_key[l] << 9;
    const int64_t node = (int64_t)(pre[l] + flag[l]) - 1;
    const uint32_t n1 = (uint32_t)((k >> 9) & 4095);
    if (flag[l]) l1_o[node] = make_int4(key_coord(k, 0) & ~127, key_coord(k, 1) & ~127, key_coord(k, 2) & ~127, 0);
    atomicOr((unsigned long long*)&l1_child[node * 64 + (n1 >> 6)], 1ull << (n1 & 63));
  }
}

unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)); }

// Stable sort of (key, pos) by all 64 key bits; the result is back in (key, pos).
void radix_sort(uint64_t* key, uint32_t* pos, int64_t n, hipStream_t st) {
  if (n <= 1) return;
  const int64_t n_tiles = (n + RS_TILE - 1) / RS_TILE;
  DevBuf<uint64_t> key2, hist, off;
  DevBuf<uint32_t> pos2;
  key2.alloc(n);
  pos2.alloc(n);
  hist.alloc(n_tiles * RS_BINS);
  off.alloc(n_tiles * RS_BINS);
  uint64_t* ka = key;
  uint64_t* kb = key2.p;
  uint32_t* pa = pos;
  uint32_t* pb = pos2.p;
  for (int pass = 0; pass < RS_PASSES; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)n_tiles), dim3(RS_THREADS), 0, st, ka, n, shift, n_tiles, hist.p);
    NVDB_HIP(hipGetLastError());
    scan_u64(hist.p, n_tiles * RS_BINS, off.p, st);
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)n_tiles), dim3(RS_THREADS), 0, st, ka, pa, n, shift, n_tiles,
                       off.p, kb, pb);
    NVDB_HIP(hipGetLastError());
    std::swap(ka, kb);
    std::swap(pa, pb);
  }
  // an even number of passes leaves the result in the caller's buffers
  static_assert(RS_PASSES % 2 == 0, "result must land in the input buffers");
  NVDB_HIP(hipStreamSynchronize(st));
}

}  // namespace

Tree* build_tree_sparse(const int32_t* ijk, const float* v, int64_t n, const nvdb_active_rule& rule, hipStream_t st) {
  NVDB_REQUIRE(n >= 0 && n < (1ll << 31), NVDB_E_INVALID, "voxel count must be in [0, 2^31)");
  NVDB_REQUIRE(n == 0 || (ijk != nullptr && v != nullptr), NVDB_E_INVALID, "null voxel arrays");
  NVDB_REQUIRE(rule.kind == NVDB_SDF || rule.kind == NVDB_FOG, NVDB_E_INVALID, "unknown active rule");
  NVDB_REQUIRE(std::isfinite(rule.band_or_threshold), NVDB_E_INVALID, "rule threshold must be finite");

  DevBuf<uint64_t> key, act, pre;
  DevBuf<uint32_t> pos;
  DevBuf<int> bad, bbox;
  key.alloc(n);
  pos.alloc(n);
  bad.alloc(1);
  bbox.alloc(6);
  const int bbox0[6] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN};
  NVDB_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), st));
  NVDB_HIP(hipMemcpyAsync(bbox.p, bbox0, sizeof(bbox0), hipMemcpyHostToDevice, st));
  int hbad = 0, hbox[6];
  std::memcpy(hbox, bbox0, sizeof(hbox));
  if (n > 0) {
    hipLaunchKernelGGL(k_sp_keys, dim3(grid_for(n)), dim3(256), 0, st, ijk, v, n, key.p, pos.p, bad.p, bbox.p);
    NVDB_HIP(hipGetLastError());
    NVDB_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
    NVDB_HIP(hipMemcpyAsync(hbox, bbox.p, sizeof(hbox), hipMemcpyDeviceToHost, st));
    NVDB_HIP(hipStreamSynchronize(st));
    NVDB_REQUIRE(!(hbad & BAD_VALUE), NVDB_E_INVALID, "voxel values contain NaN or Inf");
    NVDB_REQUIRE(!(hbad & BAD_RANGE), NVDB_E_INVALID, "voxel coordinates outside [-2^20, 2^20)");
    radix_sort(key.p, pos.p, n, st);
    act.alloc(n);
    pre.alloc(n);
    hipLaunchKernelGGL(k_sp_mark, dim3(grid_for(n)), dim3(256), 0, st, key.p, pos.p, v, n, rule.kind,
                       rule.band_or_threshold, act.p, bad.p);
    NVDB_HIP(hipGetLastError());
    NVDB_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
    NVDB_HIP(hipStreamSynchronize(st));
    NVDB_REQUIRE(!(hbad & BAD_DUPLICATE), NVDB_E_INVALID, "duplicate voxel coordinates");
  }
  const int64_t n_act = n > 0 ? (int64_t)scan_u64(act.p, n, pre.p, st) : 0;

  Tree* t = new Tree();
  try {
    for (int d = 0; d < 3; ++d) {
      t->origin[d] = n > 0 ? hbox[d] : 0;
      t->dims[d] = n > 0 ? (int32_t)std::min<int64_t>((int64_t)hbox[3 + d] - hbox[d] + 1, INT32_MAX) : 0;
    }
    t->kind = rule.kind;
    t->thr = rule.band_or_threshold;
    t->n_vox = n_act;
    DevBuf<uint64_t> ckey, lflag, lpre, leaf_key, nflag, npre;
    DevBuf<float> cval;
    if (n_act > 0) {
      ckey.alloc(n_act);
      cval.alloc(n_act);
      hipLaunchKernelGGL(k_sp_compact, dim3(grid_for(n)), dim3(256), 0, st, key.p, pos.p, v, act.p, pre.p, n, ckey.p,
                         cval.p);
      lflag.alloc(n_act);
      lpre.alloc(n_act);
      hipLaunchKernelGGL(k_sp_starts, dim3(grid_for(n_act)), dim3(256), 0, st, ckey.p, n_act, 9, lflag.p);
      NVDB_HIP(hipGetLastError());
      t->n_leaf = (int64_t)scan_u64(lflag.p, n_act, lpre.p, st);
    }
    NVDB_REQUIRE(t->n_leaf < (1ll << 23), NVDB_E_INVALID, "more than 2^23 leaves");
    t->leaf_o.alloc(std::max<int64_t>(t->n_leaf, 1));
    t->leaf_mask.alloc(std::max<int64_t>(t->n_leaf, 1) * 8);
    t->leaf_off.alloc(t->n_leaf + 1);
    t->values.alloc(std::max<int64_t>(t->n_vox, 1));
    t->vox_key.alloc(std::max<int64_t>(t->n_vox, 1));
    NVDB_HIP(hipMemsetAsync(t->leaf_mask.p, 0, t->leaf_mask.n * sizeof(uint64_t), st));
    const uint32_t nv32 = (uint32_t)t->n_vox;
    NVDB_HIP(hipMemcpyAsync(t->leaf_off.p + t->n_leaf, &nv32, sizeof(uint32_t), hipMemcpyHostToDevice, st));
    if (t->n_leaf > 0) {
      leaf_key.alloc(t->n_leaf);
      hipLaunchKernelGGL(k_sp_leaves, dim3(grid_for(n_act)), dim3(256), 0, st, ckey.p, cval.p, n_act, lflag.p, lpre.p,
                         t->leaf_o.p, t->leaf_mask.p, t->leaf_off.p, t->values.p, t->vox_key.p, leaf_key.p);
      nflag.alloc(t->n_leaf);
      npre.alloc(t->n_leaf);
      hipLaunchKernelGGL(k_sp_starts, dim3(grid_for(t->n_leaf)), dim3(256), 0, st, leaf_key.p, t->n_leaf, 12,
                         nflag.p);
      NVDB_HIP(hipGetLastError());
      t->n_l1 = (int64_t)scan_u64(nflag.p, t->n_leaf, npre.p, st);
    }
    t->l1_o.alloc(std::max<int64_t>(t->n_l1, 1));
    t->l1_child.alloc(std::max<int64_t>(t->n_l1, 1) * 64);
    t->l1_active.alloc(std::max<int64_t>(t->n_l1, 1) * 64);
    NVDB_HIP(hipMemsetAsync(t->l1_child.p, 0, t->l1_child.n * sizeof(uint64_t), st));
    NVDB_HIP(hipMemsetAsync(t->l1_active.p, 0, t->l1_active.n * sizeof(uint64_t), st));
    if (t->n_l1 > 0) {
      hipLaunchKernelGGL(k_sp_l1, dim3(grid_for(t->n_leaf)), dim3(256), 0, st, leaf_key.p, t->n_leaf, nflag.p, npre.p,
                         t->l1_o.p, t->l1_child.p);
      NVDB_HIP(hipGetLastError());
      // level-2 origins: the level-1 nodes of one level-2 node are consecutive
      std::vector<int4> l1(t->n_l1);
      NVDB_HIP(hipMemcpyAsync(l1.data(), t->l1_o.p, t->n_l1 * sizeof(int4), hipMemcpyDeviceToHost, st));
      NVDB_HIP(hipStreamSynchronize(st));
      for (const int4& o : l1) {
        const int32_t l2[3] = {o.x & ~4095, o.y & ~4095, o.z & ~4095};
        const size_t m = t->l2_origin.size();
        if (m < 3 || t->l2_origin[m - 3] != l2[0] || t->l2_origin[m - 2] != l2[1] || t->l2_origin[m - 1] != l2[2])
          t->l2_origin.insert(t->l2_origin.end(), l2, l2 + 3);
      }
    }
    t->n_l2 = (int64_t)t->l2_origin.size() / 3;
    NVDB_HIP(hipStreamSynchronize(st));
  } catch (...) {
    delete t;
    throw;
  }
  return t;
}

}  // namespace nvdb
