// Internal definitions shared by the HIP sources of libnvdb (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/nvdb.h"

namespace nvdb {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
  nvdb_status code;
  Error(nvdb_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};
#define NVDB_HIP(call)                                                                             \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      throw ::nvdb::Error(e_ == hipErrorOutOfMemory ? NVDB_E_NOMEM : NVDB_E_DEVICE,               \
                          std::string(#call) + ": " + hipGetErrorString(e_));                     \
  } while (0)
#define NVDB_REQUIRE(cond, code, msg)                                                              \
  do {                                                                                             \
    if (!(cond)) throw ::nvdb::Error(code, msg);                                                   \
  } while (0)

// ------------------------------------------------------------- vector types
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// --------------------------------------------------------- device buffers
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    NVDB_HIP(hipMalloc(&p, count * sizeof(T)));
    n = count;
  }
  void ensure(size_t count) {
    if (count > n) alloc(count);
  }
};

// ----------------------------------------------------------------- trees
struct Tree {
  int32_t origin[3], dims[3];
  int32_t kind = NVDB_SDF;     // active rule the tree was built with
  float thr = 0.f;             // its band (SDF) or threshold (fog)
  int64_t n_vox = 0, n_leaf = 0, n_l1 = 0, n_l2 = 0;
  DevBuf<int4> leaf_o;         // leaf origins (w unused)
  DevBuf<uint64_t> leaf_mask;  // [L][8]
  DevBuf<uint32_t> leaf_off;   // [L+1]
  DevBuf<float> values;        // [N] leaf-major
  DevBuf<uint32_t> vox_key;    // [N] leaf << 9 | n0
  DevBuf<int4> l1_o;           // [n_l1]
  DevBuf<uint64_t> l1_child;   // [n_l1][64]
  DevBuf<uint64_t> l1_active;  // [n_l1][64] (zero unless the tree has active tiles)
  std::vector<int32_t> l2_origin;  // host, [n_l2][3]
  int64_t n_tile = 0;          // active tiles (prune_tiles, or a decoded topology)
  DevBuf<uint32_t> tile_key;   // [n_tile] level-1 node << 12 | n1, canonical order
  DevBuf<float> tile_val;      // [n_tile]
};

// ------------------------------------------------------------- sampling
enum SampleSource : int32_t { SRC_VOXELS = 0, SRC_LEAF_SLOTS = 1, SRC_L1_SLOTS = 2, SRC_COORDS = 3, SRC_TILES = 4 };
enum LossKind : int32_t { LOSS_MSE = 0, LOSS_BCE = 1, LOSS_CE = 2, LOSS_EXTERNAL = 3 };

constexpr uint64_t SM_GOLDEN = 0x9E3779B97F4A7C15ull;
constexpr uint64_t SM_M1 = 0xBF58476D1CE4E5B9ull;
constexpr uint64_t SM_M2 = 0x94D049BB133111EBull;

// SplitMix64 output function (Steele, Lea, Flood 2014).
__host__ __device__ inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * SM_M1;
  z = (z ^ (z >> 27)) * SM_M2;
  return z ^ (z >> 31);
}
// Seed of the per-step generator: output (step+1) of the generator seeded by
// output (stream+1) of SplitMix64(seed).  Sample j of the step is output j+1
// of SplitMix64(step_seed).
inline uint64_t step_seed(uint64_t seed, int64_t stream, int64_t step) {
  uint64_t s1 = sm_mix(seed + SM_GOLDEN * (uint64_t)(stream + 1));
  return sm_mix(s1 + SM_GOLDEN * (uint64_t)(step + 1));
}

// Everything a kernel needs to turn a sample index into coordinates and targets.
struct TreeView {
  const int4* leaf_o;
  const uint64_t* leaf_mask;
  const uint32_t* vox_key;
  const float* values;
  const int4* l1_o;
  const uint64_t* l1_child;
  const uint64_t* l1_active;
  const uint32_t* tile_key;  // active tiles: level-1 node << 12 | n1
  const float* tile_val;
};

struct SampleSpec {
  int32_t src;            // SampleSource
  int32_t direct;         // sample j is population index j (decode)
  int32_t loss;           // LossKind
  uint32_t npop;          // population size for the i.i.d. sampler
  uint64_t step_seed;     // per-step SplitMix64 seed
  const uint32_t* idx;    // explicit population indices (or null)
  int64_t n;              // samples in this step / call
  float inv_n;            // 1 / n for batch-mean losses
  float tscale;           // regression target = value * tscale
  int32_t lo[3];          // normalisation box origin
  float inv_d;            // 1 / box size
  const float* coords;    // SRC_COORDS: [n][3]
  const float* gy;        // LOSS_EXTERNAL: [n][n_out]
  const uint32_t* n_dev;  // decode: optional device-side count, the samples are the first min(n, *n_dev)
  unsigned long long* bad_idx;  // explicit indices: count of indices >= npop (read as index 0), or null
};

// ----------------------------------------------------------- net layout
// Canonical parameter offsets of an H x W MLP with K inputs and C outputs.
struct NetShape {
  int32_t K, KP, W, H, C;  // KP = K rounded up to 32
  __host__ __device__ int64_t woff(int l) const {  // l = 0 .. H (H = head)
    if (l == 0) return 0;
    return (int64_t)W * K + W + (int64_t)(l - 1) * ((int64_t)W * W + W);
  }
  __host__ __device__ int64_t boff(int l) const {
    if (l == 0) return (int64_t)W * K;
    if (l == H) return woff(H) + (int64_t)C * W;
    return woff(l) + (int64_t)W * W;
  }
  __host__ __device__ int64_t nparams() const { return woff(H) + (int64_t)C * W + C; }
  __host__ __device__ int win(int l) const { return l == 0 ? K : W; }
  // floats between consecutive work-group partial gradient rows (rows start on 256-byte boundaries)
  __host__ __device__ int64_t pstride() const { return (nparams() + 63) / 64 * 64; }
};

// Device-side view of one network: FP32 master parameters are canonical; the
// kernels read "shadow" copies in their own layouts, rewritten after every
// optimiser step.
struct NetView {
  NetShape s;
  const void* wrow;      // layers 0..H-1: [W rows][256 bytes] (bf16, swizzled) or [W][Win] (fp32)
  const void* wcol;      // fp32 only: layers 0..H-1 transposed, [Win][W]
  const void* wfrag;     // bf16 only: every layer in MFMA A-fragment order (forward products)
  const void* wtfrag;    // bf16 only: layers 1..H-1 transposed, in MFMA A-fragment order (input gradients)
  const float* bias;     // [H][W]
  const float* whead;    // [C][W]
  const float* bhead;    // [C]
  const float* benc;     // feature-mapping matrix [KP/2][4] rows (bx, by, bz, 0), zero beyond n_freq
  int32_t nfreq;
  // hidden activation sin(w z) when the kernel's activation is sin:
  // w and w / (2 pi) in float and double
  float act_w, act_rev;
  double act_rev64;
};

// bf16 weight rows in LDS / HBM: 256 bytes per row (128 bf16), 8-byte chunks
// permuted by an XOR swizzle so that both the row-wise fragment reads of the
// forward product and the transposing reads of the backward product hit
// distinct LDS banks.
__host__ __device__ inline int swz(int row) { return ((row & 3) << 3) | ((row >> 2) & 7); }
__host__ __device__ inline int swz_elem(int row, int col) {  // element offset inside the row
  return (((col >> 2) ^ swz(row)) << 2) | (col & 3);
}
constexpr int ROW_ELEMS = 128;  // bf16 elements per stored row


// ----------------------------------------------------------- launch records
struct TrainNet {
  NetView net;
  TreeView tree;        // the tree this network samples
  SampleSpec spec;
  const floatx4* xt;    // gathered samples of this step: (x, y, z, target or class)
  // nonzero: the kernel draws the i.i.d. samples itself (voxels or leaf slots) from
  // the network's tree instead of reading xt
  int32_t fused;
  float* partial;       // [G][P]
  float* loss_partial;  // [G]
  // Device-side stop test (warm-started sequences): the step is skipped when
  // *prev_loss < *stop_below (both device pointers; null disables the test).
  const float* prev_loss;
  const float* stop_below;
};
// Networks of one kernel trained in one launch (gridDim.y), each on its own tree;
// the experts of a domain decomposition share launches.
constexpr int MAX_LAUNCH_NETS = 8;
struct TrainLaunch {
  TrainNet nets[MAX_LAUNCH_NETS];
  int32_t G;
};
enum InferOut : int32_t { OUT_Y = 0, OUT_VALUES = 1, OUT_MASK = 2, OUT_CLASS = 3, OUT_SCATTER = 4 };
struct InferLaunch {
  NetView net;
  SampleSpec spec;  // spec.idx null, sample j is population index j (or coordinate j)
  TreeView tree;
  int32_t out_kind;
  float out_scale;
  float* y;           // OUT_Y: [n][C]; OUT_VALUES: [n]; OUT_SCATTER: y[yidx[j]] = y_j * out_scale
  const uint32_t* yidx;
  uint64_t* mask;     // OUT_MASK: [n/64]
  uint8_t* cls;       // OUT_CLASS: [n]
  // FP8 form only: e4m3 weight fragments of every hidden layer and 1/s_w per layer
  const char* w8;
  const float* w8inv;
};
struct AdamNet {
  NetShape s;
  const float* partial;  // [G][P]
  const float* loss_partial;
  int32_t G;
  float* theta;          // FP32 master parameters, canonical
  float* m;
  float* v;
  float* grad_out;       // if non-null: write the reduced gradient and skip the update
  float* loss_out;       // if non-null: loss of this step (mean)
  float loss_scale;
  float lr, bc1, bc2;    // learning rate, 1 - beta1^s, 1 - beta2^s
  const float* prev_loss;   // stop test, as in TrainNet; a skipped step carries the loss forward
  const float* stop_below;
  int32_t* ran;             // if non-null: 1 when the step ran, 0 when skipped
  // shadow copies
  int32_t prec;
  void* wrow;
  void* wcol;
  void* wfrag;
  void* wtfrag;
  float* bias;
  float* whead;
  float* bhead;
};
// Grouped decode of many networks of one shape (the experts' forward passes).
struct GroupNet {
  NetView net;
  float out_scale;
};
struct InferGroupLaunch {
  const GroupNet* nets;         // [n_nets]
  int32_t n_nets;
  const uint32_t* chunk_start;  // [n_nets + 1]: first chunk of each network's samples, then the chunk count
  const uint32_t* count;        // [n_nets] samples per network
  const float* x;               // [chunks x chunk][3] normalised coordinates
  const uint32_t* slot;         // [chunks x chunk] output index of each sample
  float* yslot;
};
constexpr int MAX_ADAM_NETS = 16;
struct AdamLaunch {
  AdamNet nets[MAX_ADAM_NETS];
};
// One compiled decode tile shape.
struct InferVariant {
  void (*fn)(InferLaunch);
  int waves;  // waves per work-group
  int nt;     // 32-sample tiles per wave
};
constexpr int MAX_INFER_VARIANTS = 4;
struct KernelSet {
  void (*train)(TrainLaunch);          // the training kernel in use
  void (*train_classic)(TrainLaunch);  // activations in registers
  // BF16 training kernel keeping activations as LDS rows (128-wide networks on 64
  // Fourier features, one output), or null
  void (*train_rows)(TrainLaunch);
  int train_lds, infer_lds;
  void (*infer8)(InferLaunch);  // FP8 form of the forward pass
  InferVariant infer_v[MAX_INFER_VARIANTS];  // decode tile shapes, [0] the default
  int n_infer_v, infer_sel;
  void (*infer_group)(InferGroupLaunch);     // grouped decode, default tile shape
  int group_waves, group_chunk;              // its waves per work-group and samples per chunk
};
// Bytes of the e4m3 weight fragments of all hidden layers (the FP8 form).
// Elements of the bf16 fragment copies: all layers (forward), layers 1..H-1 (transposed).
__host__ __device__ inline int64_t wfrag_elems(const NetShape& s) { return (int64_t)s.W * s.KP + (int64_t)(s.H - 1) * s.W * s.W; }
__host__ __device__ inline int64_t wtfrag_elems(const NetShape& s) { return (int64_t)(s.H - 1) * s.W * s.W; }
__host__ __device__ inline int64_t fp8_weight_bytes(const NetShape& s) { return (int64_t)s.W * s.KP + (int64_t)(s.H - 1) * s.W * s.W; }

// train_rows.hip: the BF16 training kernel of the 128-wide networks keeping
// activations as LDS rows (H hidden layers), or null
void (*train_rows_kernel(int H))(TrainLaunch);
// mlp.hip
// hidden activation of a network's kernels
enum : int { ACT_RELU = 0, ACT_SIN = 1 };
bool find_kernels(int prec, int W, int H, int KP, int C, int act, KernelSet* out);
void launch_quant_fp8(const NetShape& s, const float* theta, char* w8, float* w8inv, hipStream_t st);
void launch_infer8(const KernelSet& ks, const InferLaunch& I, int grid, hipStream_t st);
void launch_train(const KernelSet& ks, const TrainLaunch& L, int n_nets, hipStream_t st);
void launch_infer_group(const KernelSet& ks, const InferGroupLaunch& M, hipStream_t st);
// work-groups of a decode launch of n samples with the selected tile shape
int infer_grid(const KernelSet& ks, int64_t n);
void launch_infer(const KernelSet& ks, const InferLaunch& I, int grid, hipStream_t st);
void launch_reduce_adam(const AdamLaunch& A, int64_t max_p, int n_nets, hipStream_t st);
void launch_write_shadow(const AdamNet& A, hipStream_t st);
void launch_sample(uint64_t sseed, uint32_t npop, int64_t n, uint32_t* out, hipStream_t st);
void launch_gather(const SampleSpec& sp, const TreeView& tv, floatx4* out, hipStream_t st);
void launch_gather_multi(const SampleSpec* sp, floatx4* const* out, int n, const TreeView& tv, hipStream_t st);
void launch_fill(float* p, int64_t n, float v, hipStream_t st);
// tree.hip
Tree* build_tree_dense(const float* grid, const int32_t dims[3], const int32_t origin[3], const nvdb_active_rule& rule,
                       hipStream_t st);
// query.hip
// Active tiles of a random access: the tree's level-1 origins and active-tile
// masks (n_l1 = 0: tiles are not looked up), and the compacted tile hits (the
// tile's normalised leaf-slot centre, the query index, the count).
struct QueryTiles {
  const int4* l1_o;
  const uint64_t* l1_active;
  int64_t n_l1;
  float* x;
  uint32_t* idx;
  uint32_t* n_hits;
};
void query_classify(const float* q, int64_t n, const Tree& tree, float background, const int32_t lo[3], float inv_d,
                    float* values, uint8_t* hits, float* hit_x, uint32_t* hit_idx, uint32_t* n_hits,
                    const QueryTiles& tiles, hipStream_t st);
// values[idx[h] C + c] = y[h C + c] * scale for the first min(n, *n_hits) rows h
void query_scatter(const float* y, const uint32_t* idx, int64_t n, const uint32_t* n_hits, float scale, float* values,
                   hipStream_t st, int C = 1);
void query_zero_count(uint32_t* c, hipStream_t st);
// Device addresses of the static scratch of the allocation-free random access on
// the current device (looked up once per device).
constexpr int64_t QUERY_NOALLOC_MAX_BATCH = 1 << 16;
struct QueryScratch {
  float* hit_x;        // [max batch][3]
  float* y;            // [max batch]
  uint32_t* hit_idx;   // [max batch]
  float* tile_x;       // [max batch][3]
  float* tile_y;       // [max batch]
  uint32_t* tile_idx;  // [max batch]
  uint32_t* cnt;       // [2]: voxel hits, tile hits
};
QueryScratch query_noalloc_scratch();
// voxels of a that b lacks, canonical order, at most cap written to out [cap][3]; returns the count
int64_t topology_patches(const Tree& a, const Tree& b, int32_t* out, int64_t cap, hipStream_t st);
// archive.hip: classes of every leaf slot of the level-1 nodes from their explicit
// child / tile masks; the tree of a decoded tree's voxels without the listed false
// positives and with the listed false negatives (device lists int32 [n][3])
void classes_from_masks(const Tree& t, uint8_t* cls, hipStream_t st);
Tree* apply_patches(const Tree& pred, const int32_t* fp, int64_t n_fp, const int32_t* fn, int64_t n_fn, hipStream_t st);
// sparse.hip
Tree* build_tree_sparse(const int32_t* ijk, const float* v, int64_t n, const nvdb_active_rule& rule, hipStream_t st);
// moe.hip: sparse domain decomposition.  Grid origin o, cell edge S, halo h, and
// the range [clo, clo + cdim) of cells a lookup table covers.
struct MoeGrid {
  int32_t o[3];
  int32_t S, h;
  int32_t clo[3];
  int32_t cdim[3];
};
struct MoeBox {  // an expert's normalisation box: x = (p - lo + 1/2) * inv_d
  int32_t lo[3];
  float inv_d;
};
constexpr int MOE_MAX_EXPERTS = 4096;
void leaf_bbox(const Tree& t, int32_t lo[3], int32_t hi[3], hipStream_t st);  // synchronises; hi exclusive
void moe_mark_cells(const Tree& t, const MoeGrid& g, uint8_t* flag, hipStream_t st);
// voxels of t inside [lo, lo + D)^3, those of its active tiles included, into ijk [n][3], v [n]
// (any order; room for n_vox + 512 n_tile); synchronises, returns the count
int64_t moe_extract(const Tree& t, const int32_t lo[3], int32_t D, int32_t* ijk, float* v, uint32_t* count,
                    hipStream_t st);
// routing and blend over the active voxels, or (slots) over every voxel slot of the leaves
// items of a blended decode: the voxels, the voxel slots of the leaves, or the
// leaf slots of the level-1 nodes
enum : int { MOE_VOXELS = 0, MOE_VOXEL_SLOTS = 1, MOE_LEAF_SLOTS = 2, MOE_TILES = 3 };
void moe_count(const Tree& t, int kind, const MoeGrid& g, const int32_t* table, int n_exp, uint32_t* cnt,
               uint32_t* uncovered, hipStream_t st);
void moe_route(const Tree& t, int kind, const MoeGrid& g, const int32_t* table, const MoeBox* box, int n_exp,
               const uint32_t* start, uint32_t* cursor, float* bx, uint32_t* bslot, uint64_t cap, hipStream_t st);
// chunk layout of the grouped decode from the per-expert counts: cs[k] first
// chunk of expert k (runs padded to whole chunks of `chunk` samples), cs[n] the
// chunk count, start[k] = cs[k] * chunk; pairs beyond cap set flag[0] (and cs[n] = 0);
// flag[1] = cnt[n] (the items no expert holds)
void moe_plan(const uint32_t* cnt, int n, int chunk, uint64_t cap, uint32_t* cs, uint32_t* start, uint32_t* flag,
              hipStream_t st);
void moe_blend(const Tree& t, int kind, const MoeGrid& g, const int32_t* table, const float* yslot, float* values,
               uint64_t* mask, uint8_t* cls, hipStream_t st);
void error_report(const Tree& t, const float* values, const uint64_t* pred_mask, nvdb_error_report* rep,
                  hipStream_t st);
void error_report_l1(const Tree& t, const uint8_t* classes, nvdb_l1_report* rep, hipStream_t st);
uint64_t scan_u64(const uint64_t* in, int64_t n, uint64_t* out, hipStream_t st);  // exclusive; returns the total
// Active tiles (tiles.hip): the pruned copy of a tree; the predicted tiles of a
// decoded topology (class-1 slots of cls, n_slots = 4096 n_l1) into t->tile_key;
// the error report over a tree's tiles.
Tree* prune_tiles(const Tree& in, hipStream_t st);
void tiles_from_classes(const uint8_t* cls, int64_t n_slots, Tree* t, hipStream_t st);
void error_report_tiles(const Tree& t, const float* pred, nvdb_error_report* rep, hipStream_t st);
void pred_flags(const uint8_t* cls, int64_t n, uint64_t* flag, hipStream_t st);
void pred_leaves(const uint8_t* cls, const uint64_t* prefix, const int4* l1_o, int64_t n, int4* leaf_o, uint64_t* child,
                 uint64_t* active, hipStream_t st);
void mask_from_values(const float* y, int64_t n_leaf, float scale, int kind, float thr, uint64_t* mask, hipStream_t st);
uint64_t pred_voxels(const uint64_t* mask, int64_t n_leaf, Tree* t, const float* slot_y, float scale, hipStream_t st);
void error_report_topology(const Tree& truth, const Tree& pred, nvdb_topology_report* rep, hipStream_t st);

}  // namespace nvdb
