// Online random access of the [Hash,5,4,NN(3)] configuration (NeuralVDB Sec. 3.5).
//
// The explicit tree decides each query: its voxel floor(q) is a hit when its
// leaf exists (binary search over the leaf origins, which are stored in the
// canonical order: level-2 origin, then n2, then n1) and the leaf's active mask
// holds it.  Hits are compacted and only they run through the regressor (whose
// launch reads the hit count on the device, so batches need no host round trip);
// every other query gets the background value.  With a tile value regressor, a
// query whose voxel lies in an active tile of a level-1 node (binary search over the
// level-1 origins, then the node's active-tile bit) is a tile hit: tile hits are
// compacted with the tile's leaf-slot centre, the tile regressor runs over them and
// they get its value, the tile's one value.  The same leaf lookup lists the
// patches of a decoded topology (voxels it adds or misses).
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "nvdb_internal.h"
#include "tree_device.h"

namespace nvdb {

// Scratch of the allocation-free random access (nvdb_query_noalloc), one copy
// per GPU for the life of the process: per query of a batch of at most
// QUERY_NOALLOC_MAX_BATCH its normalised position (3 floats), regressor output
// and query index, the same three for the tile hits, then the voxel-hit and
// tile-hit counters.  In host code `scratch` names a host stand-in, never the
// device memory: kernels get the address that hipGetSymbolAddress returns for
// the current device.
constexpr size_t QS_X = 0;
constexpr size_t QS_Y = QS_X + 12 * (size_t)QUERY_NOALLOC_MAX_BATCH;
constexpr size_t QS_IDX = QS_Y + 4 * (size_t)QUERY_NOALLOC_MAX_BATCH;
constexpr size_t QS_TX = QS_IDX + 4 * (size_t)QUERY_NOALLOC_MAX_BATCH;
constexpr size_t QS_TY = QS_TX + 12 * (size_t)QUERY_NOALLOC_MAX_BATCH;
constexpr size_t QS_TIDX = QS_TY + 4 * (size_t)QUERY_NOALLOC_MAX_BATCH;
constexpr size_t QS_CNT = QS_TIDX + 4 * (size_t)QUERY_NOALLOC_MAX_BATCH;
constexpr size_t QS_BYTES = QS_CNT + 256;
static __device__ __align__(256) char scratch[QS_BYTES];

QueryScratch query_noalloc_scratch() {
  static std::mutex mu;
  static std::map<int, char*> base;  // device -> address of its copy of `scratch`
  int dev = 0;
  NVDB_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  char*& p = base[dev];
  if (!p) {
    void* a = nullptr;
    const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !a) {
      base.erase(dev);
      throw Error(NVDB_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    p = (char*)a;
  }
  return QueryScratch{(float*)(p + QS_X),  (float*)(p + QS_Y),  (uint32_t*)(p + QS_IDX), (float*)(p + QS_TX),
                      (float*)(p + QS_TY), (uint32_t*)(p + QS_TIDX), (uint32_t*)(p + QS_CNT)};
}

namespace {

// Per query: hit test; misses get the background, hits are appended (in any
// order: each value depends only on its own query) with their normalised
// position and query index.
__global__ void __launch_bounds__(256) k_query_classify(const float* __restrict__ q, int64_t n, QueryTree t,
                                                        QueryTiles tl, float bg, int lo0, int lo1, int lo2,
                                                        float inv_d, float* __restrict__ values,
                                                        uint8_t* __restrict__ hits, float* __restrict__ hit_x,
                                                        uint32_t* __restrict__ hit_idx, uint32_t* n_hits) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float qx = q[3 * i], qy = q[3 * i + 1], qz = q[3 * i + 2];
  const float lim = 2147483648.f;  // 2^31: every float below it floors into int32
  const bool ok = isfinite(qx) && isfinite(qy) && isfinite(qz) && fabsf(qx) < lim && fabsf(qy) < lim && fabsf(qz) < lim;
  bool hit = false, in_tile = false;
  int px = 0, py = 0, pz = 0;
  if (ok) {
    px = (int)floorf(qx);
    py = (int)floorf(qy);
    pz = (int)floorf(qz);
    const int64_t a = find_leaf(t, make_int4(px & ~7, py & ~7, pz & ~7, 0));
    if (a >= 0) {
      const uint32_t n0 = (uint32_t)(((px & 7) << 6) | ((py & 7) << 3) | (pz & 7));
      hit = (t.leaf_mask[a * 8 + (n0 >> 6)] >> (n0 & 63u)) & 1ull;
    } else if (tl.n_l1 > 0) {
      const int4 o1 = make_int4(px & ~127, py & ~127, pz & ~127, 0);
      const int64_t k = lower_l1(tl.l1_o, tl.n_l1, o1);
      if (k < tl.n_l1) {
        const int4 f = tl.l1_o[k];
        if (f.x == o1.x && f.y == o1.y && f.z == o1.z) {
          const uint32_t n1 = (uint32_t)((((px >> 3) & 15) << 8) | (((py >> 3) & 15) << 4) | ((pz >> 3) & 15));
          in_tile = (tl.l1_active[k * 64 + (n1 >> 6)] >> (n1 & 63u)) & 1ull;
        }
      }
    }
  }
  if (hits) hits[i] = hit ? 1 : (in_tile ? 2 : 0);
  if (in_tile) {  // the tile's leaf-slot centre, normalised as the tile decode does it
    const uint32_t s = atomicAdd(tl.n_hits, 1u);
    tl.x[3 * (size_t)s] = ((float)((px & ~7) - lo0) + 4.f) * inv_d;
    tl.x[3 * (size_t)s + 1] = ((float)((py & ~7) - lo1) + 4.f) * inv_d;
    tl.x[3 * (size_t)s + 2] = ((float)((pz & ~7) - lo2) + 4.f) * inv_d;
    tl.idx[s] = (uint32_t)i;
    return;
  }
  if (!hit) {
    values[i] = bg;
    return;
  }
  const uint32_t s = atomicAdd(n_hits, 1u);
  hit_x[3 * (size_t)s] = (qx - (float)lo0) * inv_d;
  hit_x[3 * (size_t)s + 1] = (qy - (float)lo1) * inv_d;
  hit_x[3 * (size_t)s + 2] = (qz - (float)lo2) * inv_d;
  hit_idx[s] = (uint32_t)i;
}

__global__ void __launch_bounds__(256) k_query_scatter(const float* __restrict__ y, const uint32_t* __restrict__ idx,
                                                       int64_t n, const uint32_t* n_hits, float scale,
                                                       float* __restrict__ values, int C) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= n || h >= (int64_t)*n_hits) return;
  const size_t d = (size_t)idx[h] * C;
  for (int c = 0; c < C; ++c) values[d + c] = y[(size_t)h * C + c] * scale;
}
__global__ void k_query_zero(uint32_t* c) { *c = 0u; }

// Patches: per leaf of A, the voxels of A that B lacks (A = prediction, B = truth
// gives the false positives; the other way round the false negatives).
__global__ void __launch_bounds__(256) k_patch_count(QueryTree A, QueryTree B, uint64_t* __restrict__ cnt) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= A.n_leaf) return;
  const int64_t k = find_leaf(B, A.leaf_o[l]);
  uint64_t c = 0;
  for (int w = 0; w < 8; ++w) c += __popcll(A.leaf_mask[l * 8 + w] & ~(k >= 0 ? B.leaf_mask[k * 8 + w] : 0ull));
  cnt[l] = c;
}
__global__ void __launch_bounds__(256) k_patch_write(QueryTree A, QueryTree B, const uint64_t* __restrict__ off,
                                                     int64_t cap, int32_t* __restrict__ out) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= A.n_leaf) return;
  const int4 o = A.leaf_o[l];
  const int64_t k = find_leaf(B, o);
  int64_t s = (int64_t)off[l];
  for (int w = 0; w < 8; ++w) {
    uint64_t d = A.leaf_mask[l * 8 + w] & ~(k >= 0 ? B.leaf_mask[k * 8 + w] : 0ull);
    while (d) {
      const int n0 = 64 * w + __ffsll((long long)d) - 1;
      d &= d - 1;
      if (s < cap) {
        out[3 * s] = o.x + (n0 >> 6);
        out[3 * s + 1] = o.y + ((n0 >> 3) & 7);
        out[3 * s + 2] = o.z + (n0 & 7);
      }
      ++s;
    }
  }
}

}  // namespace

int64_t topology_patches(const Tree& a, const Tree& b, int32_t* out, int64_t cap, hipStream_t st) {
  if (a.n_leaf == 0) return 0;
  const QueryTree A{a.leaf_o.p, a.leaf_mask.p, a.n_leaf}, B{b.leaf_o.p, b.leaf_mask.p, b.n_leaf};
  DevBuf<uint64_t> cnt, off;
  cnt.alloc(a.n_leaf);
  off.alloc(a.n_leaf);
  const unsigned grid = (unsigned)((a.n_leaf + 255) / 256);
  hipLaunchKernelGGL(k_patch_count, dim3(grid), dim3(256), 0, st, A, B, cnt.p);
  NVDB_HIP(hipGetLastError());
  const int64_t total = (int64_t)scan_u64(cnt.p, a.n_leaf, off.p, st);
  if (out && cap > 0 && total > 0) {
    hipLaunchKernelGGL(k_patch_write, dim3(grid), dim3(256), 0, st, A, B, off.p, cap, out);
    NVDB_HIP(hipGetLastError());
  }
  NVDB_HIP(hipStreamSynchronize(st));
  return total;
}

void query_classify(const float* q, int64_t n, const Tree& tree, float background, const int32_t lo[3], float inv_d,
                    float* values, uint8_t* hits, float* hit_x, uint32_t* hit_idx, uint32_t* n_hits,
                    const QueryTiles& tiles, hipStream_t st) {
  if (n <= 0) return;
  QueryTree t{tree.leaf_o.p, tree.leaf_mask.p, tree.n_leaf};
  hipLaunchKernelGGL(k_query_classify, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, q, n, t, tiles, background,
                     lo[0], lo[1], lo[2], inv_d, values, hits, hit_x, hit_idx, n_hits);
  NVDB_HIP(hipGetLastError());
}

void query_scatter(const float* y, const uint32_t* idx, int64_t n, const uint32_t* n_hits, float scale, float* values,
                   hipStream_t st, int C) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_query_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, y, idx, n, n_hits, scale,
                     values, C);
  NVDB_HIP(hipGetLastError());
}
void query_zero_count(uint32_t* c, hipStream_t st) {
  hipLaunchKernelGGL(k_query_zero, dim3(1), dim3(1), 0, st, c);
  NVDB_HIP(hipGetLastError());
}

}  // namespace nvdb
