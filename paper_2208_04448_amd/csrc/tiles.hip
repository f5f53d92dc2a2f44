// Active tiles at level 1 (NeuralVDB Sec. 3.3.1): a level-1 entry may hold one
// value for a whole leaf-sized region instead of a leaf; the level-1 classifier's
// second class marks such entries and the tile value regressor encodes their
// values.  A tree built from voxels has none; prune_tiles turns every leaf whose
// 512 voxels are all active and bit-identical into an active tile, and
// tiles_from_classes lists the active tiles a decoded topology predicts.
#include <algorithm>
#include <memory>

#include "nvdb_internal.h"
#include "tree_device.h"

namespace nvdb {

// One wave per leaf: tile[i] = 1 iff its mask is full and its 512 values share one
// bit pattern (a full leaf's values are contiguous at off[i]); keep[i] = 1 - tile[i].
__global__ void __launch_bounds__(256) k_tile_flags(const uint64_t* mask, const uint32_t* off, const float* values,
                                                    int64_t n_leaf, uint64_t* tile, uint64_t* keep) {
  const int64_t leaf = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (leaf >= n_leaf) return;  // uniform per wave
  const bool word_full = lane < 8 ? mask[leaf * 8 + lane] == ~0ull : true;
  const bool full = __all(word_full);
  bool same = false;
  if (full) {
    const uint32_t* v = (const uint32_t*)(values + off[leaf]);
    const uint32_t v0 = v[0];
    bool eq = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) eq = eq && v[lane + 64 * k] == v0;
    same = __all(eq);
  }
  if (lane == 0) {
    tile[leaf] = (full && same) ? 1ull : 0ull;
    keep[leaf] = (full && same) ? 0ull : 1ull;
  }
}

// Per leaf: a kept leaf moves to its compacted place with its voxel offset
// lowered by 512 per tile before it; a tile leaf becomes tile pre_tile[i] of its
// level-1 node (child bit cleared, active-tile bit set).
__global__ void k_prune_leaves(const int4* leaf_o, const uint64_t* mask, const uint32_t* off, const float* values,
                               int64_t n_leaf, const uint64_t* tile, const uint64_t* pre_tile,
                               const uint64_t* pre_keep, const int4* l1_o, int64_t n_l1, int4* o_new,
                               uint64_t* mask_new, uint32_t* off_new, uint32_t* tile_key, float* tile_val,
                               uint64_t* l1_child, uint64_t* l1_active) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_leaf) return;
  const int4 o = leaf_o[i];
  if (tile[i]) {
    const int4 lo = make_int4(o.x & ~127, o.y & ~127, o.z & ~127, 0);
    const int64_t node = lower_l1(l1_o, n_l1, lo);
    const uint32_t n1 = (uint32_t)((((o.x >> 3) & 15) << 8) | (((o.y >> 3) & 15) << 4) | ((o.z >> 3) & 15));
    const uint64_t t = pre_tile[i];
    tile_key[t] = ((uint32_t)node << 12) | n1;
    tile_val[t] = values[off[i]];
    atomicAnd((unsigned long long*)&l1_child[node * 64 + (n1 >> 6)], ~(1ull << (n1 & 63u)));
    atomicOr((unsigned long long*)&l1_active[node * 64 + (n1 >> 6)], 1ull << (n1 & 63u));
  } else {
    const uint64_t j = pre_keep[i];
    o_new[j] = o;
#pragma unroll
    for (int w = 0; w < 8; ++w) mask_new[j * 8 + w] = mask[i * 8 + w];
    off_new[j] = off[i] - 512u * (uint32_t)pre_tile[i];
  }
}

// Per voxel of a kept leaf: its compacted place, key and value.
__global__ void k_prune_voxels(const uint32_t* vox_key, const float* values, int64_t n_vox, const uint64_t* tile,
                               const uint64_t* pre_tile, const uint64_t* pre_keep, uint32_t* key_new,
                               float* val_new) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_vox) return;
  const uint32_t key = vox_key[v], leaf = key >> 9;
  if (tile[leaf]) return;
  const int64_t nv = v - 512 * (int64_t)pre_tile[leaf];
  key_new[nv] = ((uint32_t)pre_keep[leaf] << 9) | (key & 511u);
  val_new[nv] = values[v];
}

static unsigned blocks(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

Tree* prune_tiles(const Tree& in, hipStream_t st) {
  NVDB_REQUIRE(in.n_tile == 0, NVDB_E_INVALID, "the tree already has active tiles");
  NVDB_REQUIRE(in.n_l1 < (1ll << 20), NVDB_E_INVALID, "too many level-1 nodes for 32-bit tile keys");
  std::unique_ptr<Tree> t(new Tree());
  for (int d = 0; d < 3; ++d) {
    t->origin[d] = in.origin[d];
    t->dims[d] = in.dims[d];
  }
  t->kind = in.kind;
  t->thr = in.thr;
  t->n_l1 = in.n_l1;
  t->n_l2 = in.n_l2;
  t->l2_origin = in.l2_origin;
  const int64_t nl1 = std::max<int64_t>(in.n_l1, 1);
  t->l1_o.alloc(nl1);
  t->l1_child.alloc(nl1 * 64);
  t->l1_active.alloc(nl1 * 64);
  if (in.n_l1 > 0) {
    NVDB_HIP(hipMemcpyAsync(t->l1_o.p, in.l1_o.p, in.n_l1 * sizeof(int4), hipMemcpyDeviceToDevice, st));
    NVDB_HIP(hipMemcpyAsync(t->l1_child.p, in.l1_child.p, in.n_l1 * 64 * 8, hipMemcpyDeviceToDevice, st));
    NVDB_HIP(hipMemcpyAsync(t->l1_active.p, in.l1_active.p, in.n_l1 * 64 * 8, hipMemcpyDeviceToDevice, st));
  }
  const int64_t L = in.n_leaf;
  DevBuf<uint64_t> tile, keep, pre_tile, pre_keep;
  tile.alloc(std::max<int64_t>(L, 1));
  keep.alloc(std::max<int64_t>(L, 1));
  pre_tile.alloc(std::max<int64_t>(L, 1));
  pre_keep.alloc(std::max<int64_t>(L, 1));
  if (L > 0) {
    hipLaunchKernelGGL(k_tile_flags, dim3(blocks(L, 4)), dim3(256), 0, st, in.leaf_mask.p, in.leaf_off.p, in.values.p,
                       L, tile.p, keep.p);
    NVDB_HIP(hipGetLastError());
  }
  const int64_t nt = (int64_t)scan_u64(tile.p, L, pre_tile.p, st);
  const int64_t nk = (int64_t)scan_u64(keep.p, L, pre_keep.p, st);
  NVDB_REQUIRE(nt + nk == L, NVDB_E_STATE, "tile flags inconsistent");
  t->n_tile = nt;
  t->n_leaf = nk;
  t->n_vox = in.n_vox - 512 * nt;
  t->leaf_o.alloc(std::max<int64_t>(nk, 1));
  t->leaf_mask.alloc(std::max<int64_t>(nk, 1) * 8);
  t->leaf_off.alloc(nk + 1);
  t->values.alloc(std::max<int64_t>(t->n_vox, 1));
  t->vox_key.alloc(std::max<int64_t>(t->n_vox, 1));
  t->tile_key.alloc(std::max<int64_t>(nt, 1));
  t->tile_val.alloc(std::max<int64_t>(nt, 1));
  if (L > 0) {
    hipLaunchKernelGGL(k_prune_leaves, dim3(blocks(L, 256)), dim3(256), 0, st, in.leaf_o.p, in.leaf_mask.p,
                       in.leaf_off.p, in.values.p, L, tile.p, pre_tile.p, pre_keep.p, t->l1_o.p, in.n_l1,
                       t->leaf_o.p, t->leaf_mask.p, t->leaf_off.p, t->tile_key.p, t->tile_val.p, t->l1_child.p,
                       t->l1_active.p);
    NVDB_HIP(hipGetLastError());
  }
  if (in.n_vox > 0) {
    hipLaunchKernelGGL(k_prune_voxels, dim3(blocks(in.n_vox, 256)), dim3(256), 0, st, in.vox_key.p, in.values.p,
                       in.n_vox, tile.p, pre_tile.p, pre_keep.p, t->vox_key.p, t->values.p);
    NVDB_HIP(hipGetLastError());
  }
  const uint32_t nv32 = (uint32_t)t->n_vox;
  NVDB_HIP(hipMemcpyAsync(t->leaf_off.p + nk, &nv32, sizeof(uint32_t), hipMemcpyHostToDevice, st));
  NVDB_HIP(hipStreamSynchronize(st));
  return t.release();
}

__global__ void k_class_flags(const uint8_t* cls, int64_t n, uint8_t c, uint64_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = cls[i] == c ? 1ull : 0ull;
}
__global__ void k_tile_keys(const uint64_t* flag, const uint64_t* prefix, int64_t n, uint32_t* tile_key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) tile_key[prefix[i]] = (uint32_t)i;  // slot i = node * 4096 + n1
}

void tiles_from_classes(const uint8_t* cls, int64_t n_slots, Tree* t, hipStream_t st) {
  NVDB_REQUIRE(n_slots < (1ll << 32), NVDB_E_INVALID, "too many level-1 slots for 32-bit tile keys");
  DevBuf<uint64_t> flag, prefix;
  flag.alloc(std::max<int64_t>(n_slots, 1));
  prefix.alloc(std::max<int64_t>(n_slots, 1));
  if (n_slots > 0) {
    hipLaunchKernelGGL(k_class_flags, dim3(blocks(n_slots, 256)), dim3(256), 0, st, cls, n_slots, (uint8_t)1, flag.p);
    NVDB_HIP(hipGetLastError());
  }
  const int64_t nt = (int64_t)scan_u64(flag.p, n_slots, prefix.p, st);
  t->n_tile = nt;
  t->tile_key.alloc(std::max<int64_t>(nt, 1));
  t->tile_val.alloc(std::max<int64_t>(nt, 1));
  if (n_slots > 0) {
    hipLaunchKernelGGL(k_tile_keys, dim3(blocks(n_slots, 256)), dim3(256), 0, st, flag.p, prefix.p, n_slots,
                       t->tile_key.p);
    NVDB_HIP(hipGetLastError());
  }
  NVDB_HIP(hipStreamSynchronize(st));
}

}  // namespace nvdb
