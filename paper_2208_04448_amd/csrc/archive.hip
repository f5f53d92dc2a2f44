// Compact serialised NeuralVDB (Sec. 3.3.2: the upper tree levels stay explicit,
// the lower levels are networks; Sec. 4: the networks are stored at 16 bits;
// Tab. memory_cost: 12 bytes per patch coordinate).  The byte image and the
// device work of reading it back: explicit level-1 classes, the voxel list of
// a decoded tree, and the patch application that restores the true topology.
#include <cstring>

#include "nvdb_internal.h"
#include "tree_device.h"

namespace nvdb {

namespace {

// Class of every leaf slot of the level-1 nodes from explicitly stored masks:
// 0 child leaf, 1 active tile, 2 inactive tile.
__global__ void __launch_bounds__(256) k_cls_from_masks(const uint64_t* __restrict__ child,
                                                        const uint64_t* __restrict__ active, int64_t n,
                                                        uint8_t* __restrict__ cls) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint64_t bit = 1ull << (s & 63);
  cls[s] = (child[s >> 6] & bit) ? 0 : ((active[s >> 6] & bit) ? 1 : 2);
}

// Coordinates of every voxel of a tree in its voxel order.
__global__ void __launch_bounds__(256) k_voxel_coords(const uint32_t* __restrict__ key, const int4* __restrict__ leaf_o,
                                                      int64_t n, int32_t* __restrict__ ijk) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint32_t k = key[v], n0 = k & 511u;
  const int4 o = leaf_o[k >> 9];
  ijk[3 * v] = o.x + (int)(n0 >> 6);
  ijk[3 * v + 1] = o.y + (int)((n0 >> 3) & 7u);
  ijk[3 * v + 2] = o.z + (int)(n0 & 7u);
}

// Marks the voxels of `t` listed in p[n][3]; a listed voxel that `t` lacks, or one
// listed twice, counts in *bad.
__global__ void __launch_bounds__(256) k_mark_voxels(QueryTree t, const uint32_t* __restrict__ leaf_off,
                                                     const int32_t* __restrict__ p, int64_t n,
                                                     uint32_t* __restrict__ mark, uint32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = p[3 * i], y = p[3 * i + 1], z = p[3 * i + 2];
  const int64_t leaf = find_leaf(t, make_int4(x & ~7, y & ~7, z & ~7, 0));
  const uint32_t n0 = (uint32_t)(((x & 7) << 6) | ((y & 7) << 3) | (z & 7));
  if (leaf < 0 || !((t.leaf_mask[leaf * 8 + (n0 >> 6)] >> (n0 & 63u)) & 1ull)) {
    atomicAdd(bad, 1u);
    return;
  }
  uint32_t idx = leaf_off[leaf];
  for (uint32_t w = 0; w < (n0 >> 6); ++w) idx += (uint32_t)__popcll(t.leaf_mask[leaf * 8 + w]);
  idx += (uint32_t)__popcll(t.leaf_mask[leaf * 8 + (n0 >> 6)] & ((1ull << (n0 & 63u)) - 1ull));
  if (atomicExch(&mark[idx], 1u) != 0u) atomicAdd(bad, 1u);
}

// Appends the unmarked voxels' coordinates to out (any order; the tree build sorts).
__global__ void __launch_bounds__(256) k_keep_unmarked(const int32_t* __restrict__ ijk, const uint32_t* __restrict__ mark,
                                                       int64_t n, int32_t* __restrict__ out, uint32_t* count) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || mark[v]) return;
  const uint32_t s = atomicAdd(count, 1u);
  out[3 * (size_t)s] = ijk[3 * v];
  out[3 * (size_t)s + 1] = ijk[3 * v + 1];
  out[3 * (size_t)s + 2] = ijk[3 * v + 2];
}

unsigned grid_of(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void classes_from_masks(const Tree& t, uint8_t* cls, hipStream_t st) {
  const int64_t n = 4096 * t.n_l1;
  if (n == 0) return;
  hipLaunchKernelGGL(k_cls_from_masks, dim3(grid_of(n)), dim3(256), 0, st, t.l1_child.p, t.l1_active.p, n, cls);
  NVDB_HIP(hipGetLastError());
}

Tree* apply_patches(const Tree& pred, const int32_t* fp, int64_t n_fp, const int32_t* fn, int64_t n_fn, hipStream_t st) {
  NVDB_REQUIRE(n_fp <= pred.n_vox && pred.n_vox - n_fp + n_fn < (1ll << 31), NVDB_E_INVALID,
               "patch lists do not fit the decoded tree");
  const int64_t n = pred.n_vox, n_out = n - n_fp + n_fn;
  DevBuf<int32_t> ijk, out;
  DevBuf<uint32_t> mark, cnt;
  ijk.alloc(3 * std::max<int64_t>(n, 1));
  out.alloc(3 * std::max<int64_t>(n_out, 1));
  mark.alloc(std::max<int64_t>(n, 1));
  cnt.alloc(2);
  NVDB_HIP(hipMemsetAsync(mark.p, 0, mark.n * 4, st));
  NVDB_HIP(hipMemsetAsync(cnt.p, 0, 8, st));
  if (n > 0) {
    hipLaunchKernelGGL(k_voxel_coords, dim3(grid_of(n)), dim3(256), 0, st, pred.vox_key.p, pred.leaf_o.p, n, ijk.p);
    NVDB_HIP(hipGetLastError());
  }
  if (n_fp > 0) {
    const QueryTree q{pred.leaf_o.p, pred.leaf_mask.p, pred.n_leaf};
    hipLaunchKernelGGL(k_mark_voxels, dim3(grid_of(n_fp)), dim3(256), 0, st, q, pred.leaf_off.p, fp, n_fp, mark.p,
                       cnt.p + 1);
    NVDB_HIP(hipGetLastError());
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_keep_unmarked, dim3(grid_of(n)), dim3(256), 0, st, ijk.p, mark.p, n, out.p, cnt.p);
    NVDB_HIP(hipGetLastError());
  }
  uint32_t h[2] = {0, 0};
  NVDB_HIP(hipMemcpyAsync(h, cnt.p, 8, hipMemcpyDeviceToHost, st));
  NVDB_HIP(hipStreamSynchronize(st));
  NVDB_REQUIRE(h[1] == 0 && (int64_t)h[0] == n - n_fp, NVDB_E_INVALID,
               "false-positive patch voxels missing from the decoded tree or listed twice");
  if (n_fn > 0)
    NVDB_HIP(hipMemcpyAsync(out.p + 3 * (size_t)(n - n_fp), fn, 12 * (size_t)n_fn, hipMemcpyDeviceToDevice, st));
  DevBuf<float> zero;
  zero.alloc(std::max<int64_t>(n_out, 1));
  NVDB_HIP(hipMemsetAsync(zero.p, 0, zero.n * 4, st));
  // every listed voxel is kept (a band no finite value exceeds); a false negative
  // that the decoded tree already holds is a duplicate and fails the build
  const nvdb_active_rule keep{NVDB_SDF, 3.0e38f};
  Tree* t = build_tree_sparse(out.p, zero.p, n_out, keep, st);
  t->kind = pred.kind;
  t->thr = pred.thr;
  return t;
}

}  // namespace nvdb
