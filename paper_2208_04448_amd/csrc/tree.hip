// VDB [Hash,5,4,3] tree build and error report on the GPU (NeuralVDB Sec. 3.1, Sec. 4).
//
// The dense grid is walked in "slot space": the level-1 nodes overlapping the
// grid, in canonical order (level-2 origin, then level-1 slot n2), each
// contributing its 4096 leaf slots in n1 order.  One wave reads one leaf slot
// (64 lanes x one 8-voxel z-row each, 32-byte coalesced reads), builds its
// 512-bit active mask and counts it.  A single scan over slot space then gives
// every existing leaf its canonical index and voxel offset, so no sort is
// needed; a second pass over the existing leaves compacts the values.
#include <algorithm>
#include <cstring>

#include "nvdb_internal.h"

namespace nvdb {

__device__ __forceinline__ bool active_rule(int kind, float thr, float v) {
  return kind == NVDB_SDF ? (fabsf(v) <= thr) : (v > thr);
}

struct SlotGeom {
  const int4* cand_l1;  // candidate level-1 origins, canonical order
  int32_t org[3], dims[3];
  int32_t kind;
  float thr;
};

// One wave per leaf slot: active mask (8 words) and count.
__global__ void __launch_bounds__(256) k_leaf_scan(SlotGeom g, const float* __restrict__ grid, int64_t n_slots,
                                                   uint64_t* __restrict__ slot_mask, uint64_t* __restrict__ slot_pack,
                                                   int* __restrict__ bad) {
  __shared__ uint8_t bytes[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t s = (int64_t)blockIdx.x * 4 + w; s < n_slots; s += nwaves) {
    const int4 o1 = g.cand_l1[s >> 12];
    const int n1 = (int)(s & 4095);
    const int ox = o1.x + 8 * (n1 >> 8), oy = o1.y + 8 * ((n1 >> 4) & 15), oz = o1.z + 8 * (n1 & 15);
    const int x = ox + (lane >> 3), y = oy + (lane & 7);
    uint32_t byte = 0;
    const int gx = x - g.org[0], gy = y - g.org[1];
    if (gx >= 0 && gx < g.dims[0] && gy >= 0 && gy < g.dims[1]) {
      const float* row = grid + ((int64_t)gx * g.dims[1] + gy) * g.dims[2];
#pragma unroll
      for (int z = 0; z < 8; ++z) {
        const int gz = oz + z - g.org[2];
        if (gz >= 0 && gz < g.dims[2]) {
          const float v = row[gz];
          if (!isfinite(v)) *bad = 1;
          if (active_rule(g.kind, g.thr, v)) byte |= 1u << z;
        }
      }
    }
    bytes[w][lane] = (uint8_t)byte;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    uint64_t word = 0;
    if (lane < 8) {
#pragma unroll
      for (int b = 0; b < 8; ++b) word |= (uint64_t)bytes[w][lane * 8 + b] << (8 * b);
      slot_mask[s * 8 + lane] = word;
    }
    int cnt = __popcll(word);
    // sum the 8 word counts held by lanes 0..7
#pragma unroll
    for (int off = 4; off >= 1; off >>= 1) cnt += __shfl_down(cnt, off, 8);
    if (lane == 0) slot_pack[s] = ((uint64_t)(cnt > 0) << 32) | (uint64_t)cnt;
    __builtin_amdgcn_wave_barrier();
  }
}

// Exclusive scan of 64-bit values (3 phases).
constexpr int SCAN_BLOCK = 1024;
__global__ void __launch_bounds__(256) k_scan_sums(const uint64_t* in, int64_t n, uint64_t* sums) {
  __shared__ uint64_t red[256];
  const int64_t b0 = (int64_t)blockIdx.x * SCAN_BLOCK;
  uint64_t acc = 0;
  for (int i = threadIdx.x; i < SCAN_BLOCK; i += 256)
    if (b0 + i < n) acc += in[b0 + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}
__global__ void k_scan_sums_serial(uint64_t* sums, int64_t nb, uint64_t* total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    uint64_t acc = 0;
    for (int64_t i = 0; i < nb; ++i) {
      uint64_t v = sums[i];
      sums[i] = acc;
      acc += v;
    }
    *total = acc;
  }
}
__global__ void __launch_bounds__(256) k_scan_apply(const uint64_t* in, int64_t n, const uint64_t* sums, uint64_t* out) {
  __shared__ uint64_t part[256];
  const int64_t b0 = (int64_t)blockIdx.x * SCAN_BLOCK;
  const int t = threadIdx.x;
  uint64_t v[4], loc = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = b0 + 4 * t + k;
    v[k] = i < n ? in[i] : 0;
    loc += v[k];
  }
  part[t] = loc;
  __syncthreads();
  // Hillis-Steele inclusive scan over the 256 thread totals
  for (int off = 1; off < 256; off <<= 1) {
    uint64_t add = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  uint64_t acc = sums[blockIdx.x] + (t > 0 ? part[t - 1] : 0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = b0 + 4 * t + k;
    if (i < n) out[i] = acc;
    acc += v[k];
  }
}

// Existing leaves: origin, mask, voxel offset, slot.
__global__ void k_compact_leaves(SlotGeom g, int64_t n_slots, const uint64_t* slot_pack, const uint64_t* prefix,
                                 const uint64_t* slot_mask, int4* leaf_o, uint64_t* leaf_mask, uint32_t* leaf_off,
                                 uint32_t* leaf_slot) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_slots || (slot_pack[s] >> 32) == 0) return;
  const uint64_t li = prefix[s] >> 32;
  const int4 o1 = g.cand_l1[s >> 12];
  const int n1 = (int)(s & 4095);
  leaf_o[li] = make_int4(o1.x + 8 * (n1 >> 8), o1.y + 8 * ((n1 >> 4) & 15), o1.z + 8 * (n1 & 15), 0);
#pragma unroll
  for (int k = 0; k < 8; ++k) leaf_mask[li * 8 + k] = slot_mask[s * 8 + k];
  leaf_off[li] = (uint32_t)(prefix[s] & 0xffffffffull);
  leaf_slot[li] = (uint32_t)s;
}

// Level-1 child masks of the kept level-1 nodes, and leaf counts per candidate node.
__global__ void k_l1_child(const uint64_t* slot_pack, int64_t n_cand, const int32_t* cand_to_kept, uint64_t* l1_child) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (candidate node, word)
  if (t >= n_cand * 64) return;
  const int64_t c = t >> 6;
  const int word = (int)(t & 63);
  const int32_t k = cand_to_kept[c];
  if (k < 0) return;
  uint64_t bits = 0;
  for (int b = 0; b < 64; ++b) bits |= (uint64_t)((slot_pack[c * 4096 + word * 64 + b] >> 32) & 1ull) << b;
  l1_child[(int64_t)k * 64 + word] = bits;
}
__global__ void k_cand_counts(const uint64_t* prefix, const uint64_t* slot_pack, int64_t n_cand, uint32_t* counts) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cand) return;
  const int64_t last = c * 4096 + 4095;
  counts[c] = (uint32_t)(((prefix[last] + slot_pack[last]) >> 32) - (prefix[c * 4096] >> 32));
}

// One wave per existing leaf: compacted values and keys (leaf << 9 | n0).
__global__ void __launch_bounds__(256) k_compact_voxels(SlotGeom g, const float* __restrict__ grid, int64_t n_leaf,
                                                        const int4* leaf_o, const uint64_t* leaf_mask,
                                                        const uint32_t* leaf_off, float* values, uint32_t* vox_key) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t li = (int64_t)blockIdx.x * 4 + w; li < n_leaf; li += nwaves) {
    const int4 o = leaf_o[li];
    const uint64_t* mk = leaf_mask + li * 8;
    const int wd = lane >> 3;  // mask word holding this lane's z-row (bits 8*lane .. 8*lane+7)
    uint32_t below = 0;
    for (int k = 0; k < wd; ++k) below += __popcll(mk[k]);
    const uint64_t word = mk[wd];
    const int x = o.x + (lane >> 3), y = o.y + (lane & 7);
    const float* row = grid + ((int64_t)(x - g.org[0]) * g.dims[1] + (y - g.org[1])) * g.dims[2];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
      const int n0 = lane * 8 + z;
      const int bit = n0 & 63;
      if ((word >> bit) & 1ull) {
        const uint32_t rank = below + __popcll(word & ((1ull << bit) - 1ull));
        const uint32_t dst = leaf_off[li] + rank;
        values[dst] = row[o.z + z - g.org[2]];
        vox_key[dst] = ((uint32_t)li << 9) | (uint32_t)n0;
      }
    }
  }
}

// ----------------------------------------------------------------- host
static int floor_div(int64_t a, int64_t b) { return (int)((a >= 0) ? a / b : -((-a + b - 1) / b)); }

Tree* build_tree_dense(const float* grid, const int32_t dims[3], const int32_t origin[3], const nvdb_active_rule& rule,
                       hipStream_t st) {
  NVDB_REQUIRE(grid != nullptr, NVDB_E_INVALID, "grid pointer is null");
  for (int d = 0; d < 3; ++d) {
    NVDB_REQUIRE(dims[d] > 0, NVDB_E_INVALID, "grid dims must be positive");
    NVDB_REQUIRE((int64_t)origin[d] + dims[d] + 4096 < (int64_t)INT32_MAX && (int64_t)origin[d] - 4096 > (int64_t)INT32_MIN,
                 NVDB_E_INVALID, "grid coordinates exceed the int32 index space");
  }
  NVDB_REQUIRE((int64_t)dims[0] * dims[1] * dims[2] < (1ll << 31), NVDB_E_INVALID, "grid larger than 2^31 voxels");
  NVDB_REQUIRE(rule.kind == NVDB_SDF || rule.kind == NVDB_FOG, NVDB_E_INVALID, "unknown active rule");
  NVDB_REQUIRE(std::isfinite(rule.band_or_threshold), NVDB_E_INVALID, "rule threshold must be finite");

  // candidate level-1 nodes, canonical order (level-2 origin x, y, z, then n2)
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = floor_div(origin[d], 128);
    hi[d] = floor_div((int64_t)origin[d] + dims[d] - 1, 128);
  }
  struct Cand {
    int32_t o[3];
    int64_t key[4];
  };
  std::vector<Cand> cand;
  for (int a = lo[0]; a <= hi[0]; ++a)
    for (int b = lo[1]; b <= hi[1]; ++b)
      for (int c = lo[2]; c <= hi[2]; ++c) {
        Cand k;
        k.o[0] = a * 128;
        k.o[1] = b * 128;
        k.o[2] = c * 128;
        int32_t l2[3];
        for (int d = 0; d < 3; ++d) l2[d] = k.o[d] & ~4095;
        const int n2 = (((k.o[0] >> 7) & 31) << 10) | (((k.o[1] >> 7) & 31) << 5) | ((k.o[2] >> 7) & 31);
        k.key[0] = l2[0];
        k.key[1] = l2[1];
        k.key[2] = l2[2];
        k.key[3] = n2;
        cand.push_back(k);
      }
  std::sort(cand.begin(), cand.end(), [](const Cand& x, const Cand& y) {
    return std::lexicographical_compare(x.key, x.key + 4, y.key, y.key + 4);
  });
  const int64_t n_cand = (int64_t)cand.size();
  const int64_t n_slots = n_cand * 4096;
  NVDB_REQUIRE(n_slots < (1ll << 31), NVDB_E_INVALID, "grid spans too many level-1 nodes");

  std::vector<int4> cand_o(n_cand);
  for (int64_t i = 0; i < n_cand; ++i) cand_o[i] = make_int4(cand[i].o[0], cand[i].o[1], cand[i].o[2], 0);
  DevBuf<int4> d_cand;
  d_cand.alloc(n_cand);
  NVDB_HIP(hipMemcpyAsync(d_cand.p, cand_o.data(), n_cand * sizeof(int4), hipMemcpyHostToDevice, st));

  SlotGeom g;
  g.cand_l1 = d_cand.p;
  for (int d = 0; d < 3; ++d) {
    g.org[d] = origin[d];
    g.dims[d] = dims[d];
  }
  g.kind = rule.kind;
  g.thr = rule.band_or_threshold;

  DevBuf<uint64_t> slot_mask, slot_pack, prefix, sums, total;
  DevBuf<int> bad;
  slot_mask.alloc(n_slots * 8);
  slot_pack.alloc(n_slots);
  prefix.alloc(n_slots);
  const int64_t nb = (n_slots + SCAN_BLOCK - 1) / SCAN_BLOCK;
  sums.alloc(nb);
  total.alloc(1);
  bad.alloc(1);
  NVDB_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), st));
  const int grid_slots = (int)std::min<int64_t>((n_slots + 3) / 4, 65536);
  hipLaunchKernelGGL(k_leaf_scan, dim3(grid_slots), dim3(256), 0, st, g, grid, n_slots, slot_mask.p, slot_pack.p, bad.p);
  NVDB_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(256), 0, st, slot_pack.p, n_slots, sums.p);
  hipLaunchKernelGGL(k_scan_sums_serial, dim3(1), dim3(64), 0, st, sums.p, nb, total.p);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, st, slot_pack.p, n_slots, sums.p, prefix.p);
  NVDB_HIP(hipGetLastError());
  DevBuf<uint32_t> cand_counts;
  cand_counts.alloc(n_cand);
  hipLaunchKernelGGL(k_cand_counts, dim3((unsigned)((n_cand + 255) / 256)), dim3(256), 0, st, prefix.p, slot_pack.p,
                     n_cand, cand_counts.p);
  NVDB_HIP(hipGetLastError());
  uint64_t tot = 0;
  int hbad = 0;
  std::vector<uint32_t> counts(n_cand);
  NVDB_HIP(hipMemcpyAsync(&tot, total.p, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
  NVDB_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
  NVDB_HIP(hipMemcpyAsync(counts.data(), cand_counts.p, n_cand * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  NVDB_HIP(hipStreamSynchronize(st));
  NVDB_REQUIRE(hbad == 0, NVDB_E_INVALID, "grid contains NaN or Inf values");

  Tree* t = new Tree();
  try {
    for (int d = 0; d < 3; ++d) {
      t->origin[d] = origin[d];
      t->dims[d] = dims[d];
    }
    t->kind = rule.kind;
    t->thr = rule.band_or_threshold;
    t->n_leaf = (int64_t)(tot >> 32);
    t->n_vox = (int64_t)(tot & 0xffffffffull);
    // keep the level-1 nodes that own leaves
    std::vector<int32_t> cand_to_kept(n_cand, -1);
    std::vector<int4> kept;
    for (int64_t i = 0; i < n_cand; ++i)
      if (counts[i] > 0) {
        cand_to_kept[i] = (int32_t)kept.size();
        kept.push_back(cand_o[i]);
      }
    t->n_l1 = (int64_t)kept.size();
    for (const int4& o : kept) {
      int32_t l2[3] = {o.x & ~4095, o.y & ~4095, o.z & ~4095};
      size_t m = t->l2_origin.size();
      if (m < 3 || t->l2_origin[m - 3] != l2[0] || t->l2_origin[m - 2] != l2[1] || t->l2_origin[m - 1] != l2[2])
        t->l2_origin.insert(t->l2_origin.end(), l2, l2 + 3);
    }
    t->n_l2 = (int64_t)t->l2_origin.size() / 3;

    t->leaf_o.alloc(std::max<int64_t>(t->n_leaf, 1));
    t->leaf_mask.alloc(std::max<int64_t>(t->n_leaf, 1) * 8);
    t->leaf_off.alloc(t->n_leaf + 1);
    t->values.alloc(std::max<int64_t>(t->n_vox, 1));
    t->vox_key.alloc(std::max<int64_t>(t->n_vox, 1));
    t->l1_o.alloc(std::max<int64_t>(t->n_l1, 1));
    t->l1_child.alloc(std::max<int64_t>(t->n_l1, 1) * 64);
    t->l1_active.alloc(std::max<int64_t>(t->n_l1, 1) * 64);
    DevBuf<uint32_t> leaf_slot;
    leaf_slot.alloc(std::max<int64_t>(t->n_leaf, 1));
    DevBuf<int32_t> d_map;
    d_map.alloc(n_cand);
    NVDB_HIP(hipMemcpyAsync(d_map.p, cand_to_kept.data(), n_cand * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (t->n_l1 > 0)
      NVDB_HIP(hipMemcpyAsync(t->l1_o.p, kept.data(), t->n_l1 * sizeof(int4), hipMemcpyHostToDevice, st));
    NVDB_HIP(hipMemsetAsync(t->l1_child.p, 0, t->l1_child.n * sizeof(uint64_t), st));
    NVDB_HIP(hipMemsetAsync(t->l1_active.p, 0, t->l1_active.n * sizeof(uint64_t), st));
    const uint32_t nv32 = (uint32_t)t->n_vox;
    NVDB_HIP(hipMemcpyAsync(t->leaf_off.p + t->n_leaf, &nv32, sizeof(uint32_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_compact_leaves, dim3((unsigned)((n_slots + 255) / 256)), dim3(256), 0, st, g, n_slots,
                       slot_pack.p, prefix.p, slot_mask.p, t->leaf_o.p, t->leaf_mask.p, t->leaf_off.p, leaf_slot.p);
    hipLaunchKernelGGL(k_l1_child, dim3((unsigned)((n_cand * 64 + 255) / 256)), dim3(256), 0, st, slot_pack.p, n_cand,
                       d_map.p, t->l1_child.p);
    if (t->n_leaf > 0)
      hipLaunchKernelGGL(k_compact_voxels, dim3((unsigned)std::min<int64_t>((t->n_leaf + 3) / 4, 65536)), dim3(256), 0,
                         st, g, grid, t->n_leaf, t->leaf_o.p, t->leaf_mask.p, t->leaf_off.p, t->values.p,
                         t->vox_key.p);
    NVDB_HIP(hipGetLastError());
    NVDB_HIP(hipStreamSynchronize(st));
  } catch (...) {
    delete t;
    throw;
  }
  return t;
}

// ----------------------------------------------------------------- errors
struct ErrPartial {
  double sq;
  float max_abs;
  uint32_t inter, uni;
  uint64_t fp, fn;
};

__global__ void __launch_bounds__(256) k_err_values(const float* truth, const float* pred, int64_t n, int kind,
                                                    ErrPartial* out) {
  __shared__ double s_sq[256];
  __shared__ float s_mx[256];
  __shared__ uint32_t s_in[256], s_un[256];
  double sq = 0.0;
  float mx = 0.f;
  uint32_t inter = 0, uni = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float v = truth[i], p = pred[i];
    const double d = (double)p - (double)v;
    sq += d * d;
    mx = fmaxf(mx, fabsf(p - v));
    if (isnan(p)) mx = INFINITY;
    const bool a = v <= 0.f, b = p <= 0.f;
    inter += (a && b);
    uni += (a || b);
  }
  s_sq[threadIdx.x] = sq;
  s_mx[threadIdx.x] = mx;
  s_in[threadIdx.x] = inter;
  s_un[threadIdx.x] = uni;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) {
      s_sq[threadIdx.x] += s_sq[threadIdx.x + off];
      s_mx[threadIdx.x] = fmaxf(s_mx[threadIdx.x], s_mx[threadIdx.x + off]);
      s_in[threadIdx.x] += s_in[threadIdx.x + off];
      s_un[threadIdx.x] += s_un[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[blockIdx.x].sq = s_sq[0];
    out[blockIdx.x].max_abs = s_mx[0];
    out[blockIdx.x].inter = s_in[0];
    out[blockIdx.x].uni = s_un[0];
  }
}
__global__ void __launch_bounds__(256) k_err_masks(const uint64_t* truth, const uint64_t* pred, int64_t nwords,
                                                   ErrPartial* out) {
  __shared__ uint64_t s_fp[256], s_fn[256];
  uint64_t fp = 0, fn = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * 256) {
    fp += __popcll(pred[i] & ~truth[i]);
    fn += __popcll(~pred[i] & truth[i]);
  }
  s_fp[threadIdx.x] = fp;
  s_fn[threadIdx.x] = fn;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) {
      s_fp[threadIdx.x] += s_fp[threadIdx.x + off];
      s_fn[threadIdx.x] += s_fn[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[blockIdx.x].fp = s_fp[0];
    out[blockIdx.x].fn = s_fn[0];
  }
}

void error_report(const Tree& t, const float* values, const uint64_t* pred_mask, nvdb_error_report* rep, hipStream_t st) {
  const int nblk = 512;
  DevBuf<ErrPartial> part;
  part.alloc(nblk);
  NVDB_HIP(hipMemsetAsync(part.p, 0, nblk * sizeof(ErrPartial), st));
  std::vector<ErrPartial> h(nblk);
  rep->n = t.n_vox;
  rep->max_abs = 0;
  rep->rms = 0;
  rep->iou = 1.0;
  rep->fp = rep->fn = 0;
  if (t.n_vox > 0) {
    hipLaunchKernelGGL(k_err_values, dim3(nblk), dim3(256), 0, st, t.values.p, values, t.n_vox, t.kind, part.p);
    NVDB_HIP(hipGetLastError());
  }
  if (pred_mask && t.n_leaf > 0) {
    hipLaunchKernelGGL(k_err_masks, dim3(nblk), dim3(256), 0, st, t.leaf_mask.p, pred_mask, t.n_leaf * 8, part.p);
    NVDB_HIP(hipGetLastError());
  }
  NVDB_HIP(hipMemcpyAsync(h.data(), part.p, nblk * sizeof(ErrPartial), hipMemcpyDeviceToHost, st));
  NVDB_HIP(hipStreamSynchronize(st));
  double sq = 0.0, mx = 0.0;
  uint64_t inter = 0, uni = 0, fp = 0, fn = 0;
  for (int i = 0; i < nblk; ++i) {
    sq += h[i].sq;
    mx = std::max(mx, (double)h[i].max_abs);
    inter += h[i].inter;
    uni += h[i].uni;
    fp += h[i].fp;
    fn += h[i].fn;
  }
  rep->max_abs = mx;
  rep->rms = t.n_vox > 0 ? std::sqrt(sq / (double)t.n_vox) : 0.0;
  rep->iou = (t.kind == NVDB_SDF && uni > 0) ? (double)inter / (double)uni : 1.0;
  if (t.kind != NVDB_SDF) rep->iou = -1.0;
  rep->fp = (int64_t)fp;
  rep->fn = (int64_t)fn;
}

// The same maxima and RMS over the active tiles of a tree (no IoU, no masks).
void error_report_tiles(const Tree& t, const float* pred, nvdb_error_report* rep, hipStream_t st) {
  const int nblk = 64;
  DevBuf<ErrPartial> part;
  part.alloc(nblk);
  NVDB_HIP(hipMemsetAsync(part.p, 0, nblk * sizeof(ErrPartial), st));
  std::vector<ErrPartial> h(nblk);
  if (t.n_tile > 0) {
    hipLaunchKernelGGL(k_err_values, dim3(nblk), dim3(256), 0, st, t.tile_val.p, pred, t.n_tile, (int)NVDB_FOG, part.p);
    NVDB_HIP(hipGetLastError());
  }
  NVDB_HIP(hipMemcpyAsync(h.data(), part.p, nblk * sizeof(ErrPartial), hipMemcpyDeviceToHost, st));
  NVDB_HIP(hipStreamSynchronize(st));
  double sq = 0.0, mx = 0.0;
  for (int i = 0; i < nblk; ++i) {
    sq += h[i].sq;
    mx = std::max(mx, (double)h[i].max_abs);
  }
  rep->n = t.n_tile;
  rep->max_abs = mx;
  rep->rms = t.n_tile > 0 ? std::sqrt(sq / (double)t.n_tile) : 0.0;
  rep->iou = -1.0;
  rep->fp = rep->fn = 0;
}

// ----------------------------------------------------------------- predicted topology
uint64_t scan_u64(const uint64_t* in, int64_t n, uint64_t* out, hipStream_t st) {
  if (n == 0) return 0;
  const int64_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
  DevBuf<uint64_t> sums, total;
  sums.alloc(nb);
  total.alloc(1);
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(256), 0, st, in, n, sums.p);
  hipLaunchKernelGGL(k_scan_sums_serial, dim3(1), dim3(64), 0, st, sums.p, nb, total.p);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, st, in, n, sums.p, out);
  NVDB_HIP(hipGetLastError());
  uint64_t tot = 0;
  NVDB_HIP(hipMemcpyAsync(&tot, total.p, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
  NVDB_HIP(hipStreamSynchronize(st));
  return tot;
}

__global__ void k_pred_flags(const uint8_t* cls, int64_t n, uint64_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = cls[i] == 0 ? 1ull : 0ull;
}
// Leaf origins of the slots predicted as child leaves, in slot order (canonical
// order, since the level-1 nodes are), and the level-1 child / tile bit masks.
__global__ void k_pred_leaves(const uint8_t* cls, const uint64_t* prefix, const int4* l1_o, int64_t n, int4* leaf_o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || cls[i] != 0) return;
  const int4 o = l1_o[i >> 12];
  const int n1 = (int)(i & 4095);
  leaf_o[prefix[i]] = make_int4(o.x + 8 * (n1 >> 8), o.y + 8 * ((n1 >> 4) & 15), o.z + 8 * (n1 & 15), 0);
}
__global__ void k_pred_l1_bits(const uint8_t* cls, int64_t n_words, uint64_t* child, uint64_t* active) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= n_words) return;
  uint64_t c = 0, a = 0;
  for (int b = 0; b < 64; ++b) {
    const uint8_t k = cls[w * 64 + b];
    c |= (uint64_t)(k == 0) << b;
    a |= (uint64_t)(k == 1) << b;
  }
  child[w] = c;
  active[w] = a;
}
// Voxel masks from the regressor's value at every slot, by the volume's active rule.
__global__ void k_mask_from_values(const float* y, int64_t n_words, float scale, int kind, float thr, uint64_t* mask) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= n_words) return;
  uint64_t m = 0;
  for (int b = 0; b < 64; ++b) {
    const float v = y[w * 64 + b] * scale;
    const bool act = kind == NVDB_SDF ? fabsf(v) <= thr : v > thr;
    m |= (uint64_t)act << b;
  }
  mask[w] = m;
}
__global__ void k_leaf_counts(const uint64_t* mask, int64_t n_leaf, uint64_t* cnt) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_leaf) return;
  uint64_t c = 0;
  for (int w = 0; w < 8; ++w) c += __popcll(mask[l * 8 + w]);
  cnt[l] = c;
}
// One thread per (leaf, mask word): voxel keys (and values from slot_y, if given) of
// the word's set bits, in ascending n0.
__global__ void k_pred_voxels(const uint64_t* mask, const uint64_t* prefix, int64_t n_leaf, uint32_t* leaf_off,
                              uint32_t* vox_key, const float* slot_y, float scale, float* values) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_leaf * 8) return;
  const int64_t l = t >> 3;
  const int w = (int)(t & 7);
  uint64_t pos = prefix[l];
  for (int q = 0; q < w; ++q) pos += __popcll(mask[l * 8 + q]);
  if (w == 0) leaf_off[l] = (uint32_t)prefix[l];
  uint64_t m = mask[l * 8 + w];
  while (m) {
    const int b = __builtin_ctzll(m);
    m &= m - 1;
    const uint32_t n0 = (uint32_t)(w * 64 + b);
    vox_key[pos] = (uint32_t)(l << 9) | n0;
    if (slot_y) values[pos] = slot_y[l * 512 + n0] * scale;
    ++pos;
  }
}

void pred_flags(const uint8_t* cls, int64_t n, uint64_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_pred_flags, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, cls, n, flag);
  NVDB_HIP(hipGetLastError());
}
void pred_leaves(const uint8_t* cls, const uint64_t* prefix, const int4* l1_o, int64_t n, int4* leaf_o, uint64_t* child,
                 uint64_t* active, hipStream_t st) {
  hipLaunchKernelGGL(k_pred_leaves, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, cls, prefix, l1_o, n, leaf_o);
  hipLaunchKernelGGL(k_pred_l1_bits, dim3((unsigned)((n / 64 + 255) / 256)), dim3(256), 0, st, cls, n / 64, child,
                     active);
  NVDB_HIP(hipGetLastError());
}
void mask_from_values(const float* y, int64_t n_leaf, float scale, int kind, float thr, uint64_t* mask, hipStream_t st) {
  const int64_t nw = n_leaf * 8;
  hipLaunchKernelGGL(k_mask_from_values, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, y, nw, scale, kind, thr,
                     mask);
  NVDB_HIP(hipGetLastError());
}
uint64_t pred_voxels(const uint64_t* mask, int64_t n_leaf, Tree* t, const float* slot_y, float scale, hipStream_t st) {
  if (n_leaf == 0) {
    t->n_vox = 0;
    t->values.alloc(1);
    t->vox_key.alloc(1);
    const uint32_t zero = 0;
    NVDB_HIP(hipMemcpyAsync(t->leaf_off.p, &zero, sizeof(uint32_t), hipMemcpyHostToDevice, st));
    NVDB_HIP(hipStreamSynchronize(st));
    return 0;
  }
  DevBuf<uint64_t> cnt, prefix;
  cnt.alloc(std::max<int64_t>(n_leaf, 1));
  prefix.alloc(std::max<int64_t>(n_leaf, 1));
  hipLaunchKernelGGL(k_leaf_counts, dim3((unsigned)((n_leaf + 255) / 256)), dim3(256), 0, st, mask, n_leaf, cnt.p);
  NVDB_HIP(hipGetLastError());
  const uint64_t nv = scan_u64(cnt.p, n_leaf, prefix.p, st);
  NVDB_REQUIRE(nv < (1ull << 32), NVDB_E_INVALID, "too many predicted voxels");
  t->n_vox = (int64_t)nv;
  t->values.alloc(std::max<int64_t>(t->n_vox, 1));
  t->vox_key.alloc(std::max<int64_t>(t->n_vox, 1));
  const uint32_t nv32 = (uint32_t)nv;
  NVDB_HIP(hipMemcpyAsync(t->leaf_off.p + n_leaf, &nv32, sizeof(uint32_t), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_pred_voxels, dim3((unsigned)((n_leaf * 8 + 255) / 256)), dim3(256), 0, st, mask, prefix.p,
                     n_leaf, t->leaf_off.p, t->vox_key.p, slot_y, scale, t->values.p);
  NVDB_HIP(hipGetLastError());
  NVDB_HIP(hipStreamSynchronize(st));
  return nv;
}

// Voxel-level comparison of a predicted tree with the truth; both share the
// level-1 nodes.  One wave per level-1 slot.
struct TopoPartial {
  uint64_t fp, fn, common;
  double sq;
  float max_abs;
};
__global__ void k_node_counts(const uint64_t* child, int64_t n_l1, uint64_t* cnt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_l1) return;
  uint64_t c = 0;
  for (int w = 0; w < 64; ++w) c += __popcll(child[k * 64 + w]);
  cnt[k] = c;
}
struct TopoSide {
  const uint64_t* child;      // [n_l1][64]
  const uint64_t* node_base;  // [n_l1] first leaf of each node
  const uint64_t* mask;       // [L][8]
  const uint32_t* leaf_off;
  const float* values;
};
__device__ __forceinline__ int64_t side_leaf(const TopoSide& S, int64_t node, int n1, int lane) {
  // leaf index of slot n1: node base + child bits before n1 (lane w counts word w)
  const uint64_t word = S.child[node * 64 + lane];
  const int wsel = n1 >> 6;
  int c = lane < wsel ? __popcll(word) : (lane == wsel ? __popcll(word & ((1ull << (n1 & 63)) - 1ull)) : 0);
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
  return (int64_t)S.node_base[node] + c;
}
__global__ void __launch_bounds__(256) k_err_topology(TopoSide T, TopoSide P, int64_t n_slots, TopoPartial* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint64_t fp = 0, fn = 0, common = 0;
  double sq = 0.0;
  float mx = 0.f;
  for (int64_t s = (int64_t)blockIdx.x * 4 + wv; s < n_slots; s += (int64_t)gridDim.x * 4) {
    const int64_t node = s >> 12;
    const int n1 = (int)(s & 4095);
    const bool tb = (T.child[node * 64 + (n1 >> 6)] >> (n1 & 63)) & 1ull;
    const bool pb = (P.child[node * 64 + (n1 >> 6)] >> (n1 & 63)) & 1ull;
    if (!tb && !pb) continue;
    const int64_t tl = tb ? side_leaf(T, node, n1, lane) : -1;
    const int64_t pl = pb ? side_leaf(P, node, n1, lane) : -1;
    // lane handles voxel slots 8 lane .. 8 lane + 7 (one byte of the mask)
    const int w = lane >> 3, sh = (lane & 7) * 8;
    const uint64_t tw = tb ? T.mask[tl * 8 + w] : 0ull, pw = pb ? P.mask[pl * 8 + w] : 0ull;
    const uint32_t tm = (uint32_t)((tw >> sh) & 255ull), pm = (uint32_t)((pw >> sh) & 255ull);
    fp += __popc(pm & ~tm);
    fn += __popc(tm & ~pm);
    const uint32_t both = tm & pm;
    if (__ballot(both != 0) == 0ull) continue;
    // ranks of the lane's first bit among the leaf's voxels
    uint32_t trank = 0, prank = 0;
    for (int q = 0; q < w; ++q) {
      if (tb) trank += __popcll(T.mask[tl * 8 + q]);
      if (pb) prank += __popcll(P.mask[pl * 8 + q]);
    }
    trank += __popcll(tw & ((1ull << sh) - 1ull));
    prank += __popcll(pw & ((1ull << sh) - 1ull));
    for (int b = 0; b < 8; ++b) {
      const bool tbit = (tm >> b) & 1u, pbit = (pm >> b) & 1u;
      if (tbit && pbit) {
        const float d = P.values[P.leaf_off[pl] + prank] - T.values[T.leaf_off[tl] + trank];
        sq += (double)d * (double)d;
        mx = fmaxf(mx, fabsf(d));
        if (isnan(d)) mx = INFINITY;
        ++common;
      }
      trank += tbit;
      prank += pbit;
    }
  }
  __shared__ double s_sq[256];
  __shared__ float s_mx[256];
  __shared__ uint64_t s_fp[256], s_fn[256], s_c[256];
  s_sq[threadIdx.x] = sq;
  s_mx[threadIdx.x] = mx;
  s_fp[threadIdx.x] = fp;
  s_fn[threadIdx.x] = fn;
  s_c[threadIdx.x] = common;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) {
      s_sq[threadIdx.x] += s_sq[threadIdx.x + off];
      s_mx[threadIdx.x] = fmaxf(s_mx[threadIdx.x], s_mx[threadIdx.x + off]);
      s_fp[threadIdx.x] += s_fp[threadIdx.x + off];
      s_fn[threadIdx.x] += s_fn[threadIdx.x + off];
      s_c[threadIdx.x] += s_c[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = TopoPartial{s_fp[0], s_fn[0], s_c[0], s_sq[0], s_mx[0]};
}

void error_report_topology(const Tree& truth, const Tree& pred, nvdb_topology_report* rep, hipStream_t st) {
  std::memset(rep, 0, sizeof(*rep));
  rep->n_true = truth.n_vox;
  rep->n_pred = pred.n_vox;
  const int64_t n_l1 = truth.n_l1;
  if (n_l1 == 0) return;
  DevBuf<uint64_t> tc, pc, tb, pb;
  tc.alloc(n_l1);
  pc.alloc(n_l1);
  tb.alloc(n_l1);
  pb.alloc(n_l1);
  hipLaunchKernelGGL(k_node_counts, dim3((unsigned)((n_l1 + 255) / 256)), dim3(256), 0, st, truth.l1_child.p, n_l1, tc.p);
  hipLaunchKernelGGL(k_node_counts, dim3((unsigned)((n_l1 + 255) / 256)), dim3(256), 0, st, pred.l1_child.p, n_l1, pc.p);
  NVDB_HIP(hipGetLastError());
  scan_u64(tc.p, n_l1, tb.p, st);
  scan_u64(pc.p, n_l1, pb.p, st);
  TopoSide T{truth.l1_child.p, tb.p, truth.leaf_mask.p, truth.leaf_off.p, truth.values.p};
  TopoSide P{pred.l1_child.p, pb.p, pred.leaf_mask.p, pred.leaf_off.p, pred.values.p};
  const int nblk = 512;
  DevBuf<TopoPartial> part;
  part.alloc(nblk);
  hipLaunchKernelGGL(k_err_topology, dim3(nblk), dim3(256), 0, st, T, P, 4096 * n_l1, part.p);
  NVDB_HIP(hipGetLastError());
  std::vector<TopoPartial> h(nblk);
  NVDB_HIP(hipMemcpyAsync(h.data(), part.p, nblk * sizeof(TopoPartial), hipMemcpyDeviceToHost, st));
  NVDB_HIP(hipStreamSynchronize(st));
  double sq = 0.0, mx = 0.0;
  for (const auto& e : h) {
    rep->fp += (int64_t)e.fp;
    rep->fn += (int64_t)e.fn;
    rep->n_common += (int64_t)e.common;
    sq += e.sq;
    mx = std::max(mx, (double)e.max_abs);
  }
  rep->max_abs = mx;
  rep->rms = rep->n_common > 0 ? std::sqrt(sq / (double)rep->n_common) : 0.0;
}

// Level-1 classifier against the truth: class 0 (child leaf) iff the child bit
// is set, else 1 (active tile) iff the tile-active bit is set, else 2.
struct ErrL1Partial {
  uint64_t fp, fn, mismatch;
};
__global__ void __launch_bounds__(256) k_err_l1(const uint64_t* child, const uint64_t* active, const uint8_t* cls,
                                                int64_t n_slots, ErrL1Partial* out) {
  __shared__ uint64_t s_fp[256], s_fn[256], s_mm[256];
  uint64_t fp = 0, fn = 0, mm = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_slots; i += (int64_t)gridDim.x * 256) {
    const bool c = (child[i >> 6] >> (i & 63)) & 1ull;
    const bool a = (active[i >> 6] >> (i & 63)) & 1ull;
    const int t = c ? 0 : (a ? 1 : 2);
    const int p = cls[i];
    fp += (p == 0 && t != 0);
    fn += (p != 0 && t == 0);
    mm += (p != t);
  }
  s_fp[threadIdx.x] = fp;
  s_fn[threadIdx.x] = fn;
  s_mm[threadIdx.x] = mm;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) {
      s_fp[threadIdx.x] += s_fp[threadIdx.x + off];
      s_fn[threadIdx.x] += s_fn[threadIdx.x + off];
      s_mm[threadIdx.x] += s_mm[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = ErrL1Partial{s_fp[0], s_fn[0], s_mm[0]};
}

void error_report_l1(const Tree& t, const uint8_t* classes, nvdb_l1_report* rep, hipStream_t st) {
  const int nblk = 256;
  rep->n_slots = 4096 * t.n_l1;
  rep->fp = rep->fn = rep->mismatch = 0;
  if (t.n_l1 == 0) return;
  DevBuf<ErrL1Partial> part;
  part.alloc(nblk);
  hipLaunchKernelGGL(k_err_l1, dim3(nblk), dim3(256), 0, st, t.l1_child.p, t.l1_active.p, classes, 4096 * t.n_l1,
                     part.p);
  NVDB_HIP(hipGetLastError());
  std::vector<ErrL1Partial> h(nblk);
  NVDB_HIP(hipMemcpyAsync(h.data(), part.p, nblk * sizeof(ErrL1Partial), hipMemcpyDeviceToHost, st));
  NVDB_HIP(hipStreamSynchronize(st));
  for (const auto& e : h) {
    rep->fp += (int64_t)e.fp;
    rep->fn += (int64_t)e.fn;
    rep->mismatch += (int64_t)e.mismatch;
  }
}

}  // namespace nvdb
