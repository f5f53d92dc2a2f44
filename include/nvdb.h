/*
 * libnvdb -- MI355X (gfx950) implementation of the coordinate-MLP encode/decode
 * of NeuralVDB (Kim et al., "NeuralVDB: High-resolution Sparse Volume
 * Representation using Hierarchical Neural Networks", arXiv 2208.04448).
 *
 * The calls follow the paper's problem statement: a VDB tree is built from a
 * sparse grid (Sec. 3.1), neural networks are fitted to its lower levels
 * ("encoding", Sec. 3.2-3.3), and the grid is reconstructed by inference
 * ("decoding", Sec. 3.5), with the quality measures of Sec. 4.
 *
 * Conventions for every entry point
 *   - Return value: NVDB_OK (0) or a negative nvdb_status; on failure
 *     nvdb_last_error() returns a message for the calling thread.  No C++
 *     exception and no abort crosses this boundary.
 *   - Pointers named *_dev are device (HBM) pointers; all others are host.
 *     The caller owns every pointer it passes; the library copies inputs it
 *     keeps.  Output buffers are caller-allocated, sized from the *_info /
 *     *_param_count calls.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls returning
 *     results in host memory synchronise that stream; calls writing only
 *     device buffers are asynchronous on it.
 *   - Tree handles are immutable after creation and may be shared between
 *     threads; a model handle must not be used by two threads at once.
 */
#ifndef NVDB_H
#define NVDB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nvdb_status;
enum {
  NVDB_OK = 0,
  NVDB_E_INVALID = -1,      /* bad argument, shape or input value                  */
  NVDB_E_NOMEM = -2,        /* device or host allocation failed                    */
  NVDB_E_DEVICE = -3,       /* a HIP runtime call failed                           */
  NVDB_E_NUMERIC = -4,      /* non-finite loss during a fit                        */
  NVDB_E_STATE = -5,        /* handle not in a state that allows the call          */
  NVDB_E_UNSUPPORTED = -6   /* network shape or precision without a kernel         */
};

/* Message of the last failing call on this thread ("" if none). */
const char* nvdb_last_error(void);
/* ABI version of this header (increments on incompatible changes): 2. */
int32_t nvdb_abi_version(void);

typedef struct nvdb_tree nvdb_tree;
typedef struct nvdb_model nvdb_model;

/* ------------------------------------------------------------------ trees */
/* Active-voxel rule (Sec. 3.2.1): a narrow-band level set keeps |v| <= band
 * (closed interval), a fog volume keeps v > threshold. */
enum { NVDB_SDF = 0, NVDB_FOG = 1 };
typedef struct {
  int32_t kind;             /* NVDB_SDF or NVDB_FOG */
  float band_or_threshold;  /* SDF half-width in voxels, or fog threshold */
} nvdb_active_rule;

typedef struct {
  int64_t n_voxels;         /* active voxels N                              */
  int64_t n_leaves;         /* level-0 nodes L (8^3 voxels)                 */
  int64_t n_l1;             /* level-1 nodes (16^3 leaf slots)              */
  int64_t n_l2;             /* level-2 nodes (32^3 level-1 slots)           */
  int32_t grid_origin[3];   /* index-space origin of the source grid        */
  int32_t grid_dims[3];     /* extent of the source grid                    */
  int64_t bytes_l2, bytes_l1, bytes_leaf_masks, bytes_voxels; /* Tab. memory_cost accounting */
  int64_t n_tiles;          /* active tiles at level 1 (nvdb_tree_prune_tiles) */
} nvdb_tree_info;

/* Build the [Hash,5,4,3] tree (Sec. 3.1) of a dense grid resident in HBM.
 * grid_dev: float32, dims[0]*dims[1]*dims[2] values, x-major (z fastest);
 * voxel (i,j,k) of the grid has index-space coordinate origin + (i,j,k).
 * Coordinates are decomposed bit-exactly: leaf origin p & ~7, slot
 * n0 = (x&7)<<6|(y&7)<<3|(z&7); level-1 origin p & ~127, slot
 * n1 = ((x>>3)&15)<<8|((y>>3)&15)<<4|((z>>3)&15); level-2 origin p & ~4095.
 * Leaves are ordered by (level-2 origin x,y,z, level-1 slot, leaf slot),
 * voxels inside a leaf by n0; leaf masks keep bit n in word n>>6 at n&63.
 * Errors: E_INVALID for non-positive dims, a grid beyond 2^31 voxels or
 * coordinates beyond int32, any NaN/Inf in the grid, or an unknown rule;
 * E_NOMEM / E_DEVICE from HIP.  The call synchronises `stream`. */
nvdb_status nvdb_tree_build_dense(const float* grid_dev, const int32_t dims[3], const int32_t origin[3],
                                  const nvdb_active_rule* rule, void* stream, nvdb_tree** out);
/* Build the same tree from a sparse voxel list resident in HBM: ijk_dev
 * int32[n][3] index-space coordinates, values_dev float32[n], in any order.
 * The active rule keeps the voxels it accepts (as for a dense grid); the tree
 * arrays are those nvdb_tree_build_dense produces for the same active set.
 * grid_origin / grid_dims of the tree are the bounding box of all n input
 * voxels (zero for n = 0).  Coordinates must lie in [-2^20, 2^20) (level-2
 * node index in 9 signed bits: the voxels are put in canonical order by a
 * radix sort of a 63-bit key).
 * Errors: E_INVALID for n outside [0, 2^31), null arrays with n > 0, NaN/Inf
 * values, coordinates out of range, duplicate coordinates (active or not),
 * more than 2^23 leaves, or an unknown rule; E_NOMEM / E_DEVICE from HIP.
 * Synchronises `stream`. */
nvdb_status nvdb_tree_build_sparse(const int32_t* ijk_dev, const float* values_dev, int64_t n,
                                   const nvdb_active_rule* rule, void* stream, nvdb_tree** out);
/* Counts, bounding grid and byte accounting of a tree. */
nvdb_status nvdb_tree_get_info(const nvdb_tree* tree, nvdb_tree_info* info);
/* Active tiles (Sec. 3.3.1: the level-1 entries that hold one value for a whole
 * leaf-sized region, whose values the tile value regressor encodes).  Returns a
 * new tree (free with nvdb_tree_free) in which every leaf of `in` whose 512
 * voxels are all active and bit-equal is replaced by an active tile of its
 * level-1 node: the leaf and its voxels leave the leaf and voxel arrays (the
 * rest keep their canonical order), the tile's child bit is cleared and its
 * active-tile bit set; level-1 and upper nodes are unchanged.  Tiles are kept in
 * canonical order, (level-1 node, n1); a tree without full constant leaves yields
 * a copy without tiles.  Synchronises `stream`.  Errors: E_INVALID (null
 * argument, a tree that already has tiles, 2^20 or more level-1 nodes). */
nvdb_status nvdb_tree_prune_tiles(const nvdb_tree* in, void* stream, nvdb_tree** out);
/* The active tiles of a tree to host buffers (any may be NULL): tile_key
 * uint32[T] = level-1 node index << 12 | n1, tile_value float32[T], l1_active
 * uint64[n_l1][64] (bit n1 of node k in word n1>>6 at n1&63). */
nvdb_status nvdb_tree_export_tiles(const nvdb_tree* tree, uint32_t* tile_key, float* tile_value, uint64_t* l1_active);
/* Copy the canonical arrays to host buffers (any may be NULL):
 * leaf_origin int32[L][3], leaf_mask uint64[L][8], leaf_off uint32[L+1]
 * (exclusive prefix of active counts), values float32[N] (leaf-major, n0
 * ascending), l1_origin int32[n_l1][3], l1_child uint64[n_l1][64]. */
nvdb_status nvdb_tree_export(const nvdb_tree* tree, int32_t* leaf_origin, uint64_t* leaf_mask,
                             uint32_t* leaf_off, float* values, int32_t* l1_origin, uint64_t* l1_child);
/* Upper levels (Sec. 3.1): l2_origin int32[n_l2][3] (the root's keys, in
 * canonical order) and l2_child uint64[n_l2][512], bit n2 set for every
 * level-1 node of the level-2 node (n2 = ((x>>7)&31)<<10|((y>>7)&31)<<5|((z>>7)&31)
 * of the level-1 origin).  Either may be NULL. */
nvdb_status nvdb_tree_export_l2(const nvdb_tree* tree, int32_t* l2_origin, uint64_t* l2_child);
void nvdb_tree_free(nvdb_tree* tree);

/* ----------------------------------------------------------------- models */
/* Networks of a NeuralVDB (Sec. 3.2, 3.3.1): the voxel-value regressor
 * (MSE, eq. mse), the level-0 active-mask classifier (binary cross-entropy),
 * the level-1 node classifier (three-class cross-entropy: child, active tile,
 * inactive tile) and the tile value regressor (MSE over the active tiles at
 * their leaf-slot centres, target scaled as the voxel regressor's). */
enum { NVDB_NET_REGRESSOR = 0, NVDB_NET_L0 = 1, NVDB_NET_L1 = 2, NVDB_NET_TILE = 3, NVDB_MAX_NETS = 4 };
/* Arithmetic of the matrix products: FP32 (fp32 MFMA), or BF16 operands with
 * FP32 accumulation.  Master weights, moments and losses are FP32 in both. */
enum { NVDB_FP32 = 0, NVDB_BF16 = 1 };

/* An H x W MLP after the feature mapping gamma(x) = [cos 2 pi B x ; sin 2 pi B x]
 * (eq. fm) with B of shape (n_freq, 3): K = 2 n_freq inputs, H hidden ReLU
 * layers of width W, an identity head with n_out outputs.  Parameter count
 * P = K W + W + (H-1)(W^2+W) + W n_out + n_out, canonical flat layout
 * W1, b1, W2, b2, ..., W_{H+1}, b_{H+1} with each W row-major [out][in].
 * Kernels exist, with KP = max(64, K rounded up to a multiple of 32), for
 * (W, H, KP, n_out) in {(64, 3, 64, 1), (64, 4, 128, 3), (128, 4, 128, 1),
 * (128, 3, 128, 1)} in both precisions and (128, 3, 256, 1) in BF16 (as many
 * Fourier features as the width); other shapes fail with E_UNSUPPORTED. */
typedef struct {
  int32_t width;
  int32_t hidden;
  int32_t n_freq;
  int32_t n_out;
  /* Hidden activation (App. on activation functions): 0 for ReLU, w > 0 for
   * sin(w z) on every hidden layer (the appendix uses w in 1.5 .. 3).  Kernels for
   * sin exist for (W, H, KP, n_out) = (64, 3, 64, 1) in both precisions and
   * (128, 3, 256, 1) in BF16; they have no FP8 form. */
  float sin_freq;
} nvdb_net_desc;

typedef struct {
  int32_t precision;            /* NVDB_FP32 or NVDB_BF16                                   */
  int32_t has_net[NVDB_MAX_NETS];
  nvdb_net_desc net[NVDB_MAX_NETS];
  /* Normalisation box (Sec. 3.4): x = (p - domain_lo + 1/2) / domain_size for a
   * voxel p, (o - domain_lo + 4) / domain_size for the centre of the leaf at o. */
  int32_t domain_lo[3];
  int32_t domain_size;
  /* Regression targets (Sec. 3.2): v / value_scale; for a level set value_scale
   * is the band half-width, which maps the band onto [-1, 1]; 1 for fog. */
  float value_scale;
} nvdb_model_desc;

nvdb_status nvdb_model_create(const nvdb_model_desc* desc, nvdb_model** out);
nvdb_status nvdb_model_param_count(const nvdb_model* model, int32_t net, int64_t* n);
/* Parameters in the canonical flat layout, float32, host memory.  Both wait
 * for the work this model has enqueued (its last recorded event), not for the
 * whole device, and return once the copy is complete. */
nvdb_status nvdb_model_set_params(nvdb_model* model, int32_t net, const float* params, int64_t n);
nvdb_status nvdb_model_get_params(const nvdb_model* model, int32_t net, float* params, int64_t n);
/* 16-bit storage of a network (Sec. 4 stores the networks at 16 bits): the
 * canonical parameters rounded to nearest even into IEEE binary16
 * (NVDB_STORE_F16; overflow to infinity, subnormals kept) or bfloat16
 * (NVDB_STORE_BF16), host uint16[n]; set_params16 widens them exactly and
 * loads them as nvdb_model_set_params does (non-finite values are rejected). */
enum { NVDB_STORE_F16 = 0, NVDB_STORE_BF16 = 1 };
nvdb_status nvdb_model_get_params16(const nvdb_model* model, int32_t net, int32_t kind, uint16_t* dst, int64_t n);
nvdb_status nvdb_model_set_params16(nvdb_model* model, int32_t net, int32_t kind, const uint16_t* src, int64_t n);
/* Feature-mapping matrix B, float32 [n_freq][3] row-major, host memory. */
nvdb_status nvdb_model_set_encoding(nvdb_model* model, int32_t net, const float* B, int32_t n_freq);
/* Adam state (checkpoint): first and second moments (canonical layout) and
 * the number of steps taken. */
nvdb_status nvdb_model_get_opt_state(const nvdb_model* model, int32_t net, float* m, float* v, int64_t n,
                                     int64_t* step);
nvdb_status nvdb_model_set_opt_state(nvdb_model* model, int32_t net, const float* m, const float* v,
                                     int64_t n, int64_t step);
void nvdb_model_free(nvdb_model* model);

/* ------------------------------------------------------------------- fit */
/* Training schedule (Sec. 3.2; Tab. hyperparameters): Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8) with lr_s = lr * lr_decay^floor((s-1)/lr_interval)
 * for the s-th step of each network.  Samples of a step are drawn i.i.d. by
 * the counter-based SplitMix64 sampler (stream = network id) over the
 * network's population -- active voxels (regressor), all voxel slots of the
 * leaves (level-0 classifier), all leaf slots of the level-1 nodes (level-1
 * classifier) -- or, when idx_dev[net] is given, taken in order from that
 * device array of idx_count[net] population indices, `batch` per step with a
 * shorter final step (one pass = one epoch); with index lists the call
 * synchronises `stream` and fails with E_INVALID if an index was at or beyond
 * its population size (such an index is read as 0).  The loss of a step is the
 * mean over its samples. */
typedef struct {
  int32_t steps;                 /* steps to run (per trained network)                   */
  int32_t batch;                 /* samples per step, 1 .. 2^24                          */
  uint64_t seed;
  float lr, lr_decay;
  int32_t lr_interval;
  int32_t nets_mask;             /* bit n trains network n                               */
  const uint32_t* idx_dev[NVDB_MAX_NETS];  /* optional explicit sample order             */
  int64_t idx_count[NVDB_MAX_NETS];
  /* Optional host output: summed duration in ms of the training-kernel launches,
   * measured with HIP events recorded on `stream` around each launch (the call
   * then synchronises `stream`).  NULL disables the timing. */
  float* train_kernel_ms;
} nvdb_fit_desc;

/* Run `steps` steps continuing from the model's step counters.  loss_host, if
 * not NULL, receives float[NVDB_MAX_NETS][steps] batch losses (untrained
 * networks left untouched); the call then synchronises `stream`.
 * Errors: E_INVALID (bad schedule, empty population), E_STATE (parameters or
 * encoding not set), E_NUMERIC (non-finite loss; checked when losses are
 * returned). */
nvdb_status nvdb_fit(nvdb_model* model, const nvdb_tree* tree, const nvdb_fit_desc* fit, float* loss_host,
                     void* stream);

/* Fits of several independent models (the experts of a sparse domain
 * decomposition, Sec. 3.4: each subdomain's networks train on their own voxels
 * with no exchange), models[e] on trees[e], each exactly as nvdb_fit would run
 * it, with the same schedule (i.i.d. draws only).  Per step, the networks that
 * share a training kernel and a work-group count go into launches of up to 8
 * networks (each sampling its own tree), and one optimiser launch updates up to
 * 16 networks, all on `stream`; every network's result is bit-identical to its
 * own nvdb_fit.  The call returns when every fit is done.  loss_host, if not NULL, receives
 * float[n][NVDB_MAX_NETS][steps].  fit->train_kernel_ms is ignored.  Errors:
 * E_INVALID (null arguments, n outside [1, 4096], a model listed twice, explicit
 * sample orders, bad schedule), otherwise those of nvdb_fit (on an error the
 * experts may have run part of the schedule). */
nvdb_status nvdb_fit_experts(nvdb_model* const* models, const nvdb_tree* const* trees, int32_t n,
                             const nvdb_fit_desc* fit, float* loss_host, void* stream);
/* Launch-shape autotuner.  The training step splits each network's batch over
 * G work-groups (tiles of 128 samples, one partial gradient row per work-group,
 * reduced in a fixed order before Adam); G trades the reduction's traffic
 * against filling the 256 compute units.  nvdb_autotune times reps training
 * steps of `batch` samples on `tree` (the gradient is computed and discarded:
 * parameters, optimiser state and step counters are left as they were) for each
 * candidate G in {32, 64, 128, 192, 256, 320, 384, 512} not above the tile count,
 * plus the tile count itself, and keeps the fastest for later nvdb_fit,
 * nvdb_fit_sequence and nvdb_backward_dev calls on this model.  Results for a
 * given G are deterministic; another G sums the same gradient in another order.
 * nvdb_model_set_train_groups sets G directly (0 restores the default, 256).
 * Synchronises `stream`.  Errors: E_INVALID, E_STATE as nvdb_fit. */
#define NVDB_TUNE_MAX 32
/* Training kernels: activations kept in registers (every shape), or written once
 * per layer as LDS rows with the weight gradients in the accumulation registers
 * (the BF16 128-wide networks with 128 features and one output; the default there). */
enum { NVDB_TRAIN_REGISTERS = 0, NVDB_TRAIN_ROWS = 1 };
typedef struct {
  int32_t chosen_g;
  int32_t chosen_kernel;             /* NVDB_TRAIN_*                         */
  int32_t n_candidates;
  int32_t kernel[NVDB_TUNE_MAX];
  int32_t g[NVDB_TUNE_MAX];
  float ms_per_step[NVDB_TUNE_MAX];  /* train + reduce launches of one step */
} nvdb_tune_report;
nvdb_status nvdb_autotune(nvdb_model* model, const nvdb_tree* tree, int32_t nets_mask, int32_t batch, int32_t reps,
                          nvdb_tune_report* report, void* stream);
nvdb_status nvdb_model_set_train_groups(nvdb_model* model, int32_t g);
/* The training kernel of every network of the model (NVDB_TRAIN_ROWS applies to
 * the networks that have that kernel; the others keep the register kernel).
 * nvdb_autotune also chooses among the kernels (the candidates are kernel x G).
 * Both compute the same gradient up to summation order. */
nvdb_status nvdb_model_set_train_kernel(nvdb_model* model, int32_t kind);
/* Decode tile shapes.  Each network's forward pass is compiled for a few
 * (waves per work-group, 32-sample tiles per wave) shapes — BF16 (8, 2) the
 * default, (8, 1), (4, 2), (4, 4); FP32 (8, 1) the default, (4, 1), (4, 2) —
 * which give bit-identical outputs.  nvdb_autotune_decode times reps decodes of
 * each network in nets_mask over its population of `tree` (all voxels, voxel slots
 * of the leaves, or leaf slots of the level-1 nodes) for every shape and keeps the
 * fastest for every later decode, query and forward call of that network.
 * nvdb_model_set_decode_shape selects shape `index` (in the order above) directly.
 * Synchronises `stream`.  Errors: E_INVALID, E_STATE. */
typedef struct {
  int32_t n_candidates;
  int32_t net[NVDB_TUNE_MAX];
  int32_t waves[NVDB_TUNE_MAX];
  int32_t tiles[NVDB_TUNE_MAX];
  float ms[NVDB_TUNE_MAX];      /* one decode of the network's population */
  int32_t chosen[NVDB_MAX_NETS];  /* index of the chosen shape per network    */
} nvdb_decode_tune_report;
nvdb_status nvdb_autotune_decode(nvdb_model* model, const nvdb_tree* tree, int32_t nets_mask, int32_t reps,
                                 nvdb_decode_tune_report* report, void* stream);
nvdb_status nvdb_model_set_decode_shape(nvdb_model* model, int32_t net, int32_t index);

/* Temporally coherent warm-start encoder for an animated sequence (Sec. 3.6).
 * Frame 0 is fitted from the model's current parameters with `cold` (the
 * target learning rate), then fitted again with `warm` (a rate up to 100x
 * smaller).  Every later frame starts from the previous frame's converged
 * weights and runs at most warm->steps steps of `warm`, ending early once a
 * step's batch loss falls below the final loss of frame 0's second pass; the
 * test is taken on the device before each step, per network, so the host never
 * waits inside the sequence.  Each pass starts from a fresh optimiser state
 * (zero moments, step counter 1) and draws i.i.d. batches with seed
 * cold->seed (frame 0, first pass) or warm->seed + f (frame f's warm pass).
 * cold and warm must select the same networks, have >= 1 step and no explicit
 * index lists.  use_graph != 0 records the schedule as HIP graphs of up to 512
 * steps each (fills, steps and per-frame copies; the stop test lives in the
 * kernels, so the graphs hold no host decision) and launches them in order on
 * `stream`.
 * Outputs (each may be NULL):
 *   reports[n_frames]  steps run per network (frame 0 counts both passes) and
 *                      the loss of the frame's last step that ran;
 *   loss_host          float[NVDB_MAX_NETS][T], T = cold->steps + n_frames *
 *                      warm->steps, batch losses in schedule order; a skipped
 *                      step repeats the loss that stopped the frame;
 *   frame_params_dev   device float[n_frames][sum of the trained networks'
 *                      parameter counts, ascending network id], the weights
 *                      after each frame in the canonical flat layout.
 * The model keeps the last frame's weights and optimiser state.  Synchronises
 * `stream`.  Errors as nvdb_fit; E_NUMERIC for a non-finite loss. */
typedef struct {
  int32_t steps_run[NVDB_MAX_NETS];
  float final_loss[NVDB_MAX_NETS];
} nvdb_frame_report;
nvdb_status nvdb_fit_sequence(nvdb_model* model, const nvdb_tree* const* frames, int32_t n_frames,
                              const nvdb_fit_desc* cold, const nvdb_fit_desc* warm, int32_t use_graph,
                              nvdb_frame_report* reports, float* loss_host, float* frame_params_dev,
                              void* stream);

/* ---------------------------------------------------------------- decode */
/* Offline sequential decode (Sec. 3.5) over the tree's topology:
 * values_dev (float32[N], leaf-major) receives the regressor output at every
 * active voxel scaled back to value units (y * value_scale); pred_mask_dev
 * (uint64[L][8], may be NULL) the level-0 classifier's masks, bit set iff the
 * logit is > 0.  Asynchronous on `stream`. */
nvdb_status nvdb_decode(const nvdb_model* model, const nvdb_tree* tree, float* values_dev, uint64_t* pred_mask_dev,
                        void* stream);
/* Level-1 classifier over every leaf slot of the tree's level-1 nodes
 * (4096 per node, leaf centres): classes_dev uint8[n_l1][4096], class = argmax
 * of the three logits (0 child, 1 active tile, 2 inactive tile), ties to the
 * lowest index.  Asynchronous. */
nvdb_status nvdb_decode_l1(const nvdb_model* model, const nvdb_tree* tree, uint8_t* classes_dev, void* stream);
/* The same two decodes in the FP8 form: every hidden layer multiplies e4m3
 * weights (one scale per layer, 448 / max|W|) by e4m3 inputs (one scale per
 * sample, 448 / max |h|) on the FP8 matrix cores with FP32 accumulation, then
 * divides by both scales, adds the bias and applies ReLU; the head runs in
 * FP32.  Conversions round to nearest even after clamping to +-448.  The e4m3
 * weights are rebuilt from the FP32 master parameters on every call (the
 * paper stores 16-bit networks, Sec. 4, and leaves lower-precision inference to
 * future work, Sec. 5; this form is that direction).  Asynchronous;
 * E_UNSUPPORTED when the network shape has no FP8 kernel. */
nvdb_status nvdb_decode_fp8(const nvdb_model* model, const nvdb_tree* tree, float* values_dev, uint64_t* pred_mask_dev,
                            void* stream);
nvdb_status nvdb_decode_l1_fp8(const nvdb_model* model, const nvdb_tree* tree, uint8_t* classes_dev, void* stream);
/* Tile value regressor at every active tile of the tree (leaf-slot centres, in
 * the tree's tile order): tile_values_dev float32[T] receives y * value_scale.
 * fp8 != 0 runs the FP8 form.  Asynchronous.  Errors: E_INVALID (no tile
 * regressor in the model), E_STATE (its parameters or encoding unset). */
nvdb_status nvdb_decode_tiles(const nvdb_model* model, const nvdb_tree* tree, int32_t fp8, float* tile_values_dev,
                              void* stream);

/* Error report (Sec. 4): max |v^ - v| and RMS over the true active voxels in
 * value units; IoU of the interiors {v <= 0} over the active set (level sets);
 * level-0 false positives / negatives against the true masks when
 * pred_mask_dev is given.  Synchronises `stream`. */
typedef struct {
  int64_t n;
  double max_abs;
  double rms;
  double iou;
  int64_t fp, fn;
} nvdb_error_report;
nvdb_status nvdb_errors(const nvdb_tree* tree, const float* values_dev, const uint64_t* pred_mask_dev,
                        nvdb_error_report* out, void* stream);
/* max |t^ - t| and RMS over the active tiles of the tree (value units) into
 * out->n, max_abs, rms (iou -1, fp = fn = 0).  Synchronises `stream`. */
nvdb_status nvdb_errors_tiles(const nvdb_tree* tree, const float* tile_values_dev, nvdb_error_report* out,
                              void* stream);
/* Full decode of the lower tree levels (Sec. 3.3, 3.5): the level-1 classifier
 * predicts, for every leaf slot of the level-1 nodes of `upper` (whose upper
 * levels are stored explicitly), which slots hold a leaf (a model without the
 * level-1 classifier takes the slots' classes from the child and tile masks
 * that `upper` stores, the [Hash,5,4,NN(3)] form); inside every
 * predicted leaf the level-0 classifier predicts the active voxels (logit > 0)
 * or, when the model has no level-0 classifier, the regressor's value at every
 * voxel slot is tested with the volume's active rule (SDF |v| <= band, fog
 * v > threshold, as `upper` was built); the regressor then gives each predicted
 * voxel its value.  The result is a new tree (free with nvdb_tree_free) with
 * the predicted leaves in canonical order, their masks, voxel values and the
 * predicted level-1 child / tile masks; it keeps every level-1 node of
 * `upper`.  With a tile value regressor in the model, every slot of the
 * active-tile class becomes an active tile of the result, in canonical order,
 * valued by that regressor at the slot's leaf centre (the top-down traversal of
 * Sec. 3.3.1); without one the result holds the active-tile bits but no tiles.  fp8 != 0 runs the networks in the FP8 form.  Synchronises `stream`.
 * Errors: E_STATE (a needed network missing or unset), E_INVALID. */
nvdb_status nvdb_decode_topology(const nvdb_model* model, const nvdb_tree* upper, int32_t fp8, nvdb_tree** out,
                                 void* stream);
/* Voxel-level comparison of a decoded tree with the truth it was decoded from
 * (same level-1 nodes): n_true / n_pred voxels, fp = predicted voxels that are
 * not active, fn = active voxels not predicted, and over the n_common voxels in
 * both, max |v^ - v| and RMS.  Synchronises `stream`. */
typedef struct {
  int64_t n_true, n_pred, fp, fn, n_common;
  double max_abs, rms;
} nvdb_topology_report;
nvdb_status nvdb_errors_topology(const nvdb_tree* truth, const nvdb_tree* pred, nvdb_topology_report* out,
                                 void* stream);

/* Patches (Sec. 3.3.1; 12 bytes a coordinate in Tab. memory_cost): the voxels
 * where a decoded topology `pred` (e.g. from nvdb_decode_topology) differs from
 * the truth: fp_dev int32[fp_cap][3] receives the predicted voxels that are not
 * active in `truth`, fn_dev int32[fn_cap][3] the active voxels `pred` misses,
 * each in canonical voxel order (lists beyond the caps are cut; the counts
 * n_fp / n_fn are always complete).  Removing the first list from `pred` and
 * adding the second restores the true active set exactly (lossless topology).
 * Synchronises `stream`.  Errors: E_INVALID (null counts, cap > 0 with a null
 * list). */
nvdb_status nvdb_topology_patches(const nvdb_tree* truth, const nvdb_tree* pred, int32_t* fp_dev, int64_t fp_cap,
                                  int32_t* fn_dev, int64_t fn_cap, int64_t* n_fp, int64_t* n_fn, void* stream);

/* ------------------------------------------- sparse domain decomposition */
/* Regular grid of cubic subdomains (Sec. 3.4, sparse domain decomposition):
 * cell c = (cx, cy, cz) has the core [origin + c size, origin + (c+1) size)
 * per axis and the widened box [origin + c size - halo, origin + (c+1) size +
 * halo) (the paper takes halo 8 and size 512 to 2048).  Every call checks
 * 1 <= halo, 2 halo <= size <= 2^24 and |origin| <= 2^24 (E_INVALID). */
typedef struct {
  int32_t origin[3];
  int32_t size;
  int32_t halo;
} nvdb_subdomains;

/* The cells whose core holds an active voxel of `tree`, or meets the 8^3 region
 * of one of its active tiles (the others are dropped, as the paper drops empty
 * subdomains), ascending in (cx, cy, cz):
 * the first min(n, cap) go to cells int32[cap][3] (host), the count n to
 * *n_cells.  Synchronises `stream`.  Errors: E_INVALID (null arguments, bad
 * grid, a tree spanning more than 2^24 candidate cells). */
nvdb_status nvdb_subdomain_cells(const nvdb_tree* tree, const nvdb_subdomains* grid, int32_t* cells, int64_t cap,
                                 int64_t* n_cells, void* stream);

/* Normalisation box of the expert of `cell` (Sec. 3.4: each subdomain's
 * network sees coordinates normalised to its own bounding box): lo[3] = the
 * widened box's lower corner origin + cell size - halo, *size = size + 2 halo;
 * an expert's model takes domain_lo = lo and domain_size = *size.  Host only.
 * Errors: E_INVALID (null arguments, bad grid, a corner outside [-2^30, 2^30]). */
nvdb_status nvdb_subdomain_box(const nvdb_subdomains* grid, const int32_t cell[3], int32_t lo[3], int32_t* size);

/* Training set of the expert of `cell`: the active voxels of `tree` inside the
 * cell's widened box, with their values, as a new tree (its arrays are those
 * of a tree built from that voxel list; it records the source's active rule).
 * The voxels of the source's active tiles count as active voxels of the tile's
 * value; for a source with active tiles the new tree is then pruned as by
 * nvdb_tree_prune_tiles, so that the tiles wholly inside the box are its active
 * tiles (a tile cut by the box leaves a leaf of the voxels inside).
 * An expert's model takes domain_lo = the widened box's lower corner and
 * domain_size = size + 2 halo (coordinates normalised to the subdomain's box).
 * The caller frees the result with nvdb_tree_free.  Synchronises `stream`.
 * Errors: E_INVALID (null arguments, bad grid, a box outside [-2^30, 2^30]). */
nvdb_status nvdb_tree_subdomain(const nvdb_tree* tree, const nvdb_subdomains* grid, const int32_t cell[3],
                                void* stream, nvdb_tree** out);

/* Blended decode (eq. moe) at the active voxels of `tree`: expert k is the
 * regressor of experts[k] and serves cell cells[k] (host int32[n_experts][3]).
 * Voxel p gets sum_k G_k E_k / sum_k G_k over the experts whose widened box
 * holds p (at most 8), with E_k the regressor at x = (p - domain_lo + 1/2) /
 * domain_size of that expert's own model, times its value_scale, and G_k the
 * clamped tent: the product over the axes of min(t, size + 2 halo - t,
 * 2 halo) / (2 halo), t the distance of the voxel centre from the lower face of
 * the widened box.  Each expert computes in its own precision.  values_dev is
 * float32[N] in the tree's voxel order (as nvdb_decode).  Experts of one network
 * shape run in one grouped launch.  Scratch (16 B per routed pair, sized for two
 * pairs per voxel and grown to the exact count when a call routes more, plus 32 B
 * per voxel, grown to the largest call) stays allocated on each device until the
 * process ends; calls on one device take turns on it.
 * Synchronises `stream`.  Errors: E_INVALID (null arguments, n_experts outside [1, 4096],
 * two experts for one cell, experts spanning more than 2^24 cells, a tree of
 * 2^29 voxels or more, or a voxel that no expert's widened box holds: then
 * values_dev is unspecified), E_STATE (an expert's regressor unset). */
nvdb_status nvdb_decode_moe(const nvdb_model* const* experts, const int32_t* cells, int32_t n_experts,
                            const nvdb_subdomains* grid, const nvdb_tree* tree, float* values_dev, void* stream);

/* The same blend for the level-0 masks (Sec. 3.4 applies the decomposition to
 * masks as well as values): expert k's level-0 classifier runs at every voxel slot
 * of the tree's leaves that its widened box holds, and slot bit = (sum_k G_k
 * logit_k / sum_k G_k > 0).  mask_dev is uint64[n_leaves][8] (as in
 * nvdb_decode).  The cell size and the grid origin must be multiples of 8 (then a
 * leaf never straddles two cores and every slot has its leaf's expert).  Scratch,
 * synchronisation and errors as nvdb_decode_moe, with 2^29 voxel slots as the
 * limit and E_STATE for an unset level-0 classifier. */
nvdb_status nvdb_decode_moe_mask(const nvdb_model* const* experts, const int32_t* cells, int32_t n_experts,
                                 const nvdb_subdomains* grid, const nvdb_tree* tree, uint64_t* mask_dev,
                                 void* stream);

/* The same blend for the level-1 classes (the decomposition applies to every
 * network of the hierarchy, Sec. 3.4): expert k's level-1 classifier runs at every
 * leaf slot of the tree's level-1 nodes that its widened box holds, at
 * x = (o - domain_lo + 4) / domain_size for the slot at origin o; the three
 * logits are blended with the gates taken at the slot's centre o + 4, and the
 * slot's class is the argmax of the blended logits (ties to the lowest class).
 * classes_dev is uint8[n_l1][4096] (as nvdb_decode_l1).  The cell size, the halo
 * and the grid origin must be multiples of 8 (a slot then lies wholly inside or
 * outside every widened box).  Experts of one network shape and precision share
 * one grouped launch; otherwise each expert runs its own.  Synchronisation,
 * scratch (96 B per leaf slot in place of 32 B per voxel) and errors as
 * nvdb_decode_moe_mask, E_STATE for an unset level-1 classifier. */
nvdb_status nvdb_decode_moe_l1(const nvdb_model* const* experts, const int32_t* cells, int32_t n_experts,
                               const nvdb_subdomains* grid, const nvdb_tree* tree, uint8_t* classes_dev,
                               void* stream);

/* The same blend for the values of active tiles (Sec. 3.3.1 tiles under the
 * decomposition of Sec. 3.4): expert k's tile value regressor runs at every
 * active tile of the tree that its widened box holds, at x = (o - domain_lo + 4)
 * / domain_size for the tile at leaf-slot origin o, times the expert's value
 * scale; the values are blended with the gates taken at the tile's centre o + 4
 * (the gates of nvdb_decode_moe_l1).  tile_values_dev is float[n_tiles] in the
 * tree's tile order (as nvdb_decode_tiles).  The cell size, the halo and the grid
 * origin must be multiples of 8.  Synchronisation, scratch (32 B per tile) and
 * errors as nvdb_decode_moe, E_STATE for an unset tile value regressor; a tree
 * without tiles returns at once. */
nvdb_status nvdb_decode_moe_tiles(const nvdb_model* const* experts, const int32_t* cells, int32_t n_experts,
                                  const nvdb_subdomains* grid, const nvdb_tree* tree, float* tile_values_dev,
                                  void* stream);

/* Level-1 classifier report (Sec. 3.3.1, Sec. 4) over the 4096 leaf slots of
 * every level-1 node: classes_dev is uint8[n_l1][4096] as written by
 * nvdb_decode_l1; the true class of a slot is 0 when it has a child leaf, else
 * 1 when it is an active tile, else 2.  fp counts slots predicted as child
 * leaves that are not, fn child leaves predicted as anything else, mismatch
 * every slot whose class differs.  Synchronises `stream`. */
typedef struct {
  int64_t n_slots;
  int64_t fp, fn, mismatch;
} nvdb_l1_report;
nvdb_status nvdb_errors_l1(const nvdb_tree* tree, const uint8_t* classes_dev, nvdb_l1_report* out, void* stream);

/* Online random access of the [Hash,5,4,NN(3)] configuration (Sec. 3.5):
 * values at n query positions q_dev float32[n][3] in index space (voxel p
 * covers [p, p+1) per axis).  The explicit tree decides each query: its voxel
 * floor(q) is a hit when the voxel's leaf exists and its active mask holds it;
 * hits get the regressor's value at q, normalised like the voxel centres
 * ((q - domain_lo) / domain_size) and scaled back by value_scale, so a query at
 * a voxel centre returns that voxel's decoded value.  When the tree has active
 * tiles (nvdb_tree_prune_tiles) and the model holds the tile value regressor, a
 * query whose voxel lies in an active tile's region gets that regressor's value
 * at the tile's leaf-slot centre (the tile's one value, bit-equal to
 * nvdb_decode_tiles).  Every other query (including non-finite positions) gets
 * `background`.  The networks run only on their hits.  Queries are processed in
 * batches of `batch` (0: all at once).  hits_dev (uint8[n], may be NULL)
 * receives 1 for regressor queries, 2 for tile queries, 0 otherwise.  Device
 * buffers; synchronises `stream`.  Errors: E_INVALID (bad buffers or sizes,
 * n >= 2^31, non-finite background), E_STATE (regressor, or the tile regressor
 * a tree with tiles needs, missing or unset). */
nvdb_status nvdb_query(const nvdb_model* model, const nvdb_tree* tree, const float* q_dev, int64_t n, float background,
                       int64_t batch, float* values_dev, uint8_t* hits_dev, void* stream);

/* nvdb_query without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, serving loops that forbid hipMalloc): the same
 * values and hit flags as nvdb_query, active tiles included, computed by the
 * same kernels, with the per-batch scratch (2.5 MiB: positions, outputs and
 * indices of the voxel hits and of the tile hits of one batch of at most 65536
 * queries, and the two hit counters) in a static device array that each GPU
 * holds until the process ends.  batch 0 means 65536; a batch above 65536 is
 * E_INVALID.  Asynchronous on `stream` (no synchronisation).  Every call on one
 * GPU shares that GPU's scratch: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller; calls on one stream
 * are ordered.  Errors as nvdb_query, E_DEVICE if the scratch's device address
 * cannot be obtained. */
nvdb_status nvdb_query_noalloc(const nvdb_model* model, const nvdb_tree* tree, const float* q_dev, int64_t n,
                               float background, int64_t batch, float* values_dev, uint8_t* hits_dev, void* stream);

/* ---------------------------------------------------------------- archive */
/* Compact serialised NeuralVDB (Sec. 3.3.2: the upper tree levels are kept
 * explicitly and the lower levels are replaced by networks; Sec. 4: networks
 * stored at 16 bits; Tab. memory_cost: 12 bytes per patch coordinate).  The byte
 * image (little-endian, sections 4-byte aligned): a 120-byte header (magic
 * "NVDB", version 1, flags, 16-bit format, the arithmetic the patches were taken
 * with, active rule, value scale, normalisation box, grid box, network mask, node,
 * patch and stored-leaf counts); per level-2 node its origin (12 B) and child
 * mask (4096 B); per level-1 node its origin (12 B) and, when the level is stored
 * explicitly, its child and tile masks (2 x 512 B); when the leaf masks are
 * stored ([Hash,5,4,NN(3)]: only the voxel values are neural), each leaf's
 * 512-bit mask (64 B) in canonical leaf order; per network
 * (regressor, level-0, level-1 classifier, those in nets_mask) its shape
 * int32[4] (width, hidden, n_freq, n_out) and sin frequency float32 (0: ReLU),
 * encoding float32[n_freq][3] and
 * parameters uint16[P] rounded to nearest even (padded to 4 bytes); then the
 * false-positive and false-negative voxel coordinates int32[n][3].
 * nvdb_archive_write: the archive of `model`'s networks for the volume `truth`
 * (stored leaf masks need stored level-1 masks, no level-0 classifier and no
 * patches: their topology is exact).
 * With patches, the writer decodes the topology the reader will decode (the
 * 16-bit networks, in the model's arithmetic, from the stored upper levels)
 * and lists where it differs from `truth`, so the reader restores the true
 * active set exactly.  cap 0 with buf NULL returns the size only.
 * A truth with active tiles is archived with its level-1 and leaf masks stored
 * (no patches): the reader's top-down decode then places the tiles exactly and
 * values them with the tile value regressor, which the archive must hold.
 * Synchronises `stream`.  Errors: E_INVALID (bad description, buffer smaller
 * than *size), E_STATE (a network missing or unset), E_UNSUPPORTED (patches
 * requested for a truth with active tiles).
 * nvdb_archive_decode: the tree decoded from an archive: the lower levels by
 * inference from the stored upper levels (nvdb_decode_topology), the patches
 * applied, values from the regressor at every voxel.  The caller frees the tree.
 * Synchronises `stream`.  Errors: E_INVALID (not an archive, truncated, corrupt
 * sizes or origins, patches that do not match the decoded tree). */
typedef struct {
  int32_t nets_mask;    /* networks stored; must hold the regressor                  */
  int32_t storage;      /* NVDB_STORE_F16 or NVDB_STORE_BF16                        */
  int32_t explicit_l1;  /* 1: level-1 child / tile masks stored (no level-1 net)    */
  int32_t patches;      /* 1: store the patches that make the topology lossless      */
  int32_t explicit_l0;  /* 1: leaf masks stored (no level-0 inference)              */
} nvdb_archive_desc;
typedef struct {
  int32_t flags;      /* bit 0: level-1 masks, bit 1: patches, bit 2: leaf masks */
  int32_t nets_mask;  /* networks stored                                     */
  int32_t rule_kind;  /* active rule of the encoded volume                   */
  float rule_thr;
  int64_t n_l2, n_l1, n_fp, n_fn, n_leaf;  /* n_leaf: leaf masks stored           */
} nvdb_archive_info;
nvdb_status nvdb_archive_write(const nvdb_model* model, const nvdb_tree* truth, const nvdb_archive_desc* desc,
                               uint8_t* buf, int64_t cap, int64_t* size, void* stream);
nvdb_status nvdb_archive_decode(const uint8_t* buf, int64_t size, nvdb_tree** out, nvdb_archive_info* info,
                                void* stream);

/* ------------------------------------------------- device-pointer calls */
/* Calls for the autograd binding and for callers that keep their own batches
 * on the device.  None of them allocates or synchronises: their workspace is
 * reserved beforehand by nvdb_model_reserve_dev, so a sequence of them can be
 * recorded into a HIP graph.  They are asynchronous on `stream`.
 *
 * nvdb_model_reserve_dev: workspace for _dev calls of network `net` on batches
 *   of up to max_n samples (partial gradient rows and gathered samples).  It
 *   allocates and synchronises; the buffers keep their addresses until the next
 *   reserve call or nvdb_model_free, so recorded graphs stay valid in between.
 *   The work-groups per training launch are fixed here (the autotuned value,
 *   else the default).  Errors: E_INVALID (max_n outside [1, 2^24]).
 *
 * The population of a network (Sec. 3.3.1) on `tree`: the regressor's is the
 *   tree's N active voxels in its voxel order, the level-0 classifier's the
 *   512 L voxel slots of its leaves (index leaf * 512 + n0), the level-1
 *   classifier's the 4096 L1 leaf slots of its level-1 nodes (node * 4096 + n1,
 *   at leaf centres).  An index is gathered and normalised inside the kernel
 *   with the model's box (Sec. 3.4): x = (p - domain_lo + 1/2) / domain_size.
 *   Indices must be below the population size: an index beyond it is read as 0
 *   and counted in the model's index-error word (nvdb_model_take_errors).
 *
 * nvdb_forward_dev: y_dev float32[n][n_out] = network outputs (normalised units,
 *   logits for classifiers) at the samples idx_dev uint32[n].
 * nvdb_backward_dev: grad_dev float32[P] (canonical layout) =
 *   sum_i sum_c gy_dev[i][c] dy_c(x_i)/dtheta over the samples idx_dev[i], the
 *   forward activations recomputed inside the fused kernel (no activation is
 *   stored).  n <= the reserved max_n (E_STATE otherwise).
 * nvdb_forward_coords_dev / nvdb_backward_coords_dev: the same at caller-given
 *   normalised coordinates x_dev float32[n][3] instead of population indices.
 * nvdb_model_set_params_dev / nvdb_model_get_params_dev: the canonical FP32
 *   parameters from / to device memory (float32[P]), ordered on `stream`; set
 *   also rewrites the kernels' weight copies.  Values are not checked for
 *   finiteness (that would need a synchronisation).
 * nvdb_sample_indices_dev: the sampler's indices idx_dev[j] = floor(h * n_pop / 2^64),
 *   h = SplitMix64 hash of (seed, stream_id, step, j), j < batch.
 * Errors of all: E_INVALID (null or oversized buffers, empty population),
 *   E_STATE (parameters or encoding unset, workspace not reserved). */
nvdb_status nvdb_model_reserve_dev(nvdb_model* model, int32_t net, int64_t max_n);
nvdb_status nvdb_forward_dev(const nvdb_model* model, int32_t net, const nvdb_tree* tree, const uint32_t* idx_dev,
                             int64_t n, float* y_dev, void* stream);
nvdb_status nvdb_backward_dev(nvdb_model* model, int32_t net, const nvdb_tree* tree, const uint32_t* idx_dev,
                              const float* gy_dev, int64_t n, float* grad_dev, void* stream);
nvdb_status nvdb_forward_coords_dev(const nvdb_model* model, int32_t net, const float* x_dev, int64_t n, float* y_dev,
                                    void* stream);
nvdb_status nvdb_backward_coords_dev(nvdb_model* model, int32_t net, const float* x_dev, const float* gy_dev,
                                     int64_t n, float* grad_dev, void* stream);
nvdb_status nvdb_model_set_params_dev(nvdb_model* model, int32_t net, const float* params_dev, int64_t n,
                                      void* stream);
nvdb_status nvdb_model_get_params_dev(const nvdb_model* model, int32_t net, float* params_dev, int64_t n,
                                      void* stream);
nvdb_status nvdb_sample_indices_dev(uint64_t seed, int32_t stream_id, int64_t step, int64_t n_pop, int64_t batch,
                                    uint32_t* idx_dev, void* stream);
/* Waits for the model's enqueued work, then returns and clears its error word:
 * *n_bad_index = number of sample indices at or beyond their population size
 * read since the last call (explicit index lists of nvdb_fit and the _dev
 * calls).  nvdb_fit with index lists checks it itself (E_INVALID). */
nvdb_status nvdb_model_take_errors(nvdb_model* model, int64_t* n_bad_index);

#ifdef __cplusplus
}
#endif
#endif /* NVDB_H */
