// Coordinate-MLP kernels of NeuralVDB for gfx950 (MI355X).
//
// What is computed (NeuralVDB, arXiv 2208.04448):
//   gamma(x) = [cos 2 pi B x ; sin 2 pi B x]                       (Sec. 3.2.2, eq. fm)
//   a_{l+1} = ReLU(W_l a_l + b_l), l < H;  y = W_H a_H + b_H        (Sec. 3.2, 3.3.1)
//   losses: MSE (eq. mse), binary and three-class cross-entropy     (Sec. 3.2, 3.3.1)
//   backward: dW_l = sum_b g_{l+1} a_l^T, g_l = (W_l^T g_{l+1}) * 1[a_l > 0]
//   Adam with a staircase exponential learning-rate decay           (Sec. 3.2, appendix)
//
// How it is laid out on CDNA4.  A wave owns 32 samples.  Every product runs on
// MFMA 32x32 tiles in the "transposed" orientation Z^T = W A^T: the weight
// fragment is the A operand and the activation tile the B operand, so the
// output tile has one sample per lane column and 16 features per lane in the
// accumulator registers.  That register layout ("S layout") is exactly the B
// operand layout of the next layer up to a fixed permutation of the input
// features inside each block of 16, which is folded into how weight fragments
// are read, so layers chain without any data movement.  The backward chain
// uses the same orientation with W^T fragments, read from the same LDS copy of
// W through the gfx950 transposing LDS load.  The weight gradients need the
// batch as the contraction dimension: each wave writes its activation and
// gradient tiles as rows to LDS and every wave reads, again with transposing
// loads, the fragments of the 32x32 blocks of dW it owns, accumulating them in
// registers for the whole step (BF16 form) or in its work-group's partial row
// in HBM (FP32 form).  A deterministic fixed-order reduction over work-groups
// then feeds Adam, which also rewrites the weight copies the kernels read.
#include "nvdb_internal.h"

namespace nvdb {

// Lane index, opaque to the optimiser: swizzled LDS addresses are functions of the
// lane, and without this the compiler hoists hundreds of them out of the
// persistent loops and keeps them live in registers.  Recomputing an address
// costs a couple of VALU operations that issue under the MFMA shadow.
__device__ __forceinline__ int lane_id() {
  int v = threadIdx.x & 63;
  asm volatile("" : "+v"(v));
  return v;
}
template <int V>
struct IC {
  static constexpr int value = V;
};
// Compile-time loop: f(IC<I>{}), f(IC<I+1>{}), ..., f(IC<N-1>{}).
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(IC<I>{});
    static_for<I + 1, N>(f);
  }
}
// A zero the compiler cannot see through.  Adding it to LDS parameter addresses
// inside the persistent loops keeps loop-invariant loads from being hoisted out
// of the loop, where they would pin hundreds of registers.
__device__ __forceinline__ int opaque_zero() {
  int z = 0;
  asm volatile("" : "+s"(z));
  return z;
}
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  bf16x2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ float shfl_xor32(float v) {
  // exchange with the lane 32 apart (other half of the wave)
  int src = (lane_id() ^ 32) << 2;
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v)));
}

// ------------------------------------------------------------ precision traits
template <int PREC>
struct PR;

template <>
struct PR<NVDB_BF16> {
  static constexpr int KS = 2;  // MFMA k-steps per 32-feature block
  static constexpr int SR = 8;  // 32-bit registers holding one S-layout block
  using Frag = bf16x8;
  static __device__ __forceinline__ floatx16 mma(Frag a, Frag b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ Frag sfrag(const uint32_t* s, int kk) {
    u32x4 v = {s[4 * kk], s[4 * kk + 1], s[4 * kk + 2], s[4 * kk + 3]};
    return __builtin_bit_cast(Frag, v);
  }
  static __device__ __forceinline__ void store(const floatx16& a, uint32_t* s) {
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] = pack_bf16x2(a[2 * i], a[2 * i + 1]);
  }
  static __device__ __forceinline__ bool positive(const uint32_t* s, int r) {
    uint32_t w = (r & 1) ? (s[r >> 1] >> 16) : (s[r >> 1] & 0xffffu);
    return w != 0u && (w & 0x8000u) == 0u;
  }
};

template <>
struct PR<NVDB_FP32> {
  static constexpr int KS = 16;
  static constexpr int SR = 16;
  using Frag = float;
  static __device__ __forceinline__ floatx16 mma(Frag a, Frag b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ Frag sfrag(const uint32_t* s, int kk) { return __uint_as_float(s[kk]); }
  static __device__ __forceinline__ void store(const floatx16& a, uint32_t* s) {
#pragma unroll
    for (int i = 0; i < 16; ++i) s[i] = __float_as_uint(a[i]);
  }
  static __device__ __forceinline__ bool positive(const uint32_t* s, int r) { return __uint_as_float(s[r]) > 0.f; }
};

// Feature held in accumulator register r (0..15) of block t by lane half h.
__device__ __forceinline__ int sfeat(int t, int r, int h) { return 32 * t + 8 * (r >> 2) + 4 * h + (r & 3); }

typedef __attribute__((address_space(3))) shortx4 lds_shortx4;
__device__ __forceinline__ u32x2 lds_tr(const __bf16* p) {
  shortx4 v = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_shortx4*)(p));
  return __builtin_bit_cast(u32x2, v);
}

// ------------------------------------------------------------------ samples
struct Smp {
  float x[3];
  float t;     // regression / binary target
  int cls;     // class label (level-1 classifier)
  bool valid;
};

__device__ __forceinline__ Smp fetch_sample(const SampleSpec& sp, const TreeView& tv, int64_t j) {
  Smp s;
  s.x[0] = s.x[1] = s.x[2] = 0.f;
  s.t = 0.f;
  s.cls = 0;
  s.valid = j < sp.n;
  if (!s.valid) return s;
  if (sp.src == SRC_COORDS) {
    s.x[0] = sp.coords[3 * j];
    s.x[1] = sp.coords[3 * j + 1];
    s.x[2] = sp.coords[3 * j + 2];
    return s;
  }
  uint32_t g;
  if (sp.direct) {
    g = (uint32_t)j;
  } else if (sp.idx) {
    g = sp.idx[j];
  } else {
    uint64_t h = sm_mix(sp.step_seed + SM_GOLDEN * (uint64_t)(j + 1));
    g = (uint32_t)__umul64hi(h, (uint64_t)sp.npop);
  }
  int px, py, pz;
  float half = 0.5f;
  if (sp.src == SRC_VOXELS) {
    uint32_t key = tv.vox_key[g];
    int4 o = tv.leaf_o[key >> 9];
    uint32_t n0 = key & 511u;
    px = o.x + (int)(n0 >> 6);
    py = o.y + (int)((n0 >> 3) & 7u);
    pz = o.z + (int)(n0 & 7u);
    s.t = tv.values[g] * sp.tscale;
  } else if (sp.src == SRC_LEAF_SLOTS) {
    uint32_t leaf = g >> 9, n0 = g & 511u;
    int4 o = tv.leaf_o[leaf];
    px = o.x + (int)(n0 >> 6);
    py = o.y + (int)((n0 >> 3) & 7u);
    pz = o.z + (int)(n0 & 7u);
    s.t = (float)((tv.leaf_mask[(size_t)leaf * 8 + (n0 >> 6)] >> (n0 & 63u)) & 1ull);
  } else {  // SRC_L1_SLOTS: leaf centres of every slot of the level-1 nodes
    uint32_t node = g >> 12, n1 = g & 4095u;
    int4 o = tv.l1_o[node];
    px = o.x + 8 * (int)(n1 >> 8);
    py = o.y + 8 * (int)((n1 >> 4) & 15u);
    pz = o.z + 8 * (int)(n1 & 15u);
    half = 4.f;
    uint64_t c = (tv.l1_child[(size_t)node * 64 + (n1 >> 6)] >> (n1 & 63u)) & 1ull;
    uint64_t a = (tv.l1_active[(size_t)node * 64 + (n1 >> 6)] >> (n1 & 63u)) & 1ull;
    s.cls = c ? 0 : (a ? 1 : 2);
  }
  s.x[0] = ((float)(px - sp.lo[0]) + half) * sp.inv_d;
  s.x[1] = ((float)(py - sp.lo[1]) + half) * sp.inv_d;
  s.x[2] = ((float)(pz - sp.lo[2]) + half) * sp.inv_d;
  return s;
}

// gamma(x) into S layout.  Feature f < m is cos(2 pi b_f.x) = sin(2 pi (b_f.x + 1/4)),
// m <= f < 2m is sin(2 pi b_{f-m}.x), f >= 2m is zero padding.  The hardware sine
// takes revolutions; the phase is reduced with fract first.  The FP32 form forms the
// phase in double precision so the feature is accurate to the sine's own error.
template <int PREC, int NIB>
__device__ __forceinline__ void encode_S(const Smp& s, const float* benc, int m, uint32_t (&X)[NIB][PR<PREC>::SR]) {
  const int h = lane_id() >> 5;
#pragma unroll
  for (int t = 0; t < NIB; ++t) {
    floatx16 v;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      int f = sfeat(t, r, h);
      int fi = f < m ? f : f - m;
      fi = fi < m ? fi : 0;
      float b0 = benc[3 * fi], b1 = benc[3 * fi + 1], b2 = benc[3 * fi + 2];
      float ph;
      if constexpr (PREC == NVDB_FP32) {
        double u = (double)b0 * s.x[0] + (double)b1 * s.x[1] + (double)b2 * s.x[2] + (f < m ? 0.25 : 0.0);
        ph = (float)(u - floor(u));
      } else {
        float u = fmaf(b0, s.x[0], fmaf(b1, s.x[1], b2 * s.x[2])) + (f < m ? 0.25f : 0.f);
        ph = __builtin_amdgcn_fractf(u);
      }
      float val = __builtin_amdgcn_sinf(ph);
      v[r] = (f < 2 * m) ? val : 0.f;
    }
    PR<PREC>::store(v, X[t]);
  }
}

// ------------------------------------------------------------ fragment loads
// bf16 weight rows are stored with 128 elements per row and swizzled 8-byte chunks.
__device__ __forceinline__ bf16x8 frag_rows_bf16(const __bf16* rows, int row, int col) {
  // elements [col, col+4) and [col+8, col+12) of `row` (col multiple of 4)
  const __bf16* base = rows + row * ROW_ELEMS;
  u32x2 a = *(const u32x2*)(base + swz_elem(row, col));
  u32x2 b = *(const u32x2*)(base + swz_elem(row, col + 8));
  u32x4 v = {a[0], a[1], b[0], b[1]};
  return __builtin_bit_cast(bf16x8, v);
}
// Transposing read: lane (i, h) receives rows rbase + 8p + 4h + e (p, e) of column cbase + i.
__device__ __forceinline__ bf16x8 frag_cols_bf16(const __bf16* rows, int rbase, int cbase) {
  const int l = lane_id(), g = l >> 4, k = l & 15, h = g >> 1, gg = g & 1;
  const int col = cbase + 16 * gg + 4 * (k & 3);
  const int r0 = rbase + 4 * h + (k >> 2);
  u32x2 a = lds_tr(rows + r0 * ROW_ELEMS + swz_elem(r0, col));
  u32x2 b = lds_tr(rows + (r0 + 8) * ROW_ELEMS + swz_elem(r0 + 8, col));
  u32x4 v = {a[0], a[1], b[0], b[1]};
  return __builtin_bit_cast(bf16x8, v);
}
// Write the lane's S-layout blocks of one sample as a row of bf16 (swizzled).
template <int NIB>
__device__ __forceinline__ void write_rows_bf16(__bf16* rows, const uint32_t (&S)[NIB][8]) {
  const int s = lane_id() & 31, h = lane_id() >> 5;
  __bf16* base = rows + s * ROW_ELEMS;
#pragma unroll
  for (int t = 0; t < NIB; ++t)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      u32x2 v = {S[t][2 * a], S[t][2 * a + 1]};
      *(u32x2*)(base + swz_elem(s, 32 * t + 8 * a + 4 * h)) = v;
    }
}
template <int NIB>
__device__ __forceinline__ void write_rows_f32(float* rows, int pitch, const uint32_t (&S)[NIB][16]) {
  const int s = lane_id() & 31, h = lane_id() >> 5;
  float* base = rows + s * pitch;
#pragma unroll
  for (int t = 0; t < NIB; ++t)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      floatx4 v = {__uint_as_float(S[t][4 * a]), __uint_as_float(S[t][4 * a + 1]), __uint_as_float(S[t][4 * a + 2]),
                   __uint_as_float(S[t][4 * a + 3])};
      *(floatx4*)(base + 32 * t + 8 * a + 4 * h) = v;
    }
}
__device__ __forceinline__ float row_elem_bf16(const __bf16* rows, int s, int f) {
  return (float)rows[s * ROW_ELEMS + swz_elem(s, f)];
}

// ------------------------------------------------------------ per-layer weights
// A fragment of W_l for the forward product: rows = output features of block ob,
// k-step kk of input block t.
template <int PREC, int W, int KP>
struct WFwd {
  const __bf16* lds;       // bf16 rows (layers >= 1 staged in LDS)
  const u32x4* gfrag;      // bf16 layer-0 fragments in HBM
  const float* gcol;       // fp32: layer transposed [Win][W] in HBM
  int layer;
  __device__ __forceinline__ typename PR<PREC>::Frag operator()(int ob, int t, int kk) const {
    if constexpr (PREC == NVDB_BF16) {
      if (layer == 0) {
        return __builtin_bit_cast(bf16x8, gfrag[((ob * (KP / 32) + t) * 2 + kk) * 64 + lane_id()]);
      }
      return frag_rows_bf16(lds, 32 * ob + (lane_id() & 31), 32 * t + 16 * kk + 4 * (lane_id() >> 5));
    } else {
      const int h = lane_id() >> 5;
      return gcol[(size_t)sfeat(t, kk, h) * W + 32 * ob + (lane_id() & 31)];
    }
  }
};
// A fragment of W_l^T for the backward product: rows = input features of block ib,
// k-step kk of output block t.
template <int PREC, int W>
struct WBwd {
  const __bf16* lds;
  const float* grow;  // fp32: [W][W] row-major
  __device__ __forceinline__ typename PR<PREC>::Frag operator()(int ib, int t, int kk) const {
    if constexpr (PREC == NVDB_BF16) {
      return frag_cols_bf16(lds, 32 * t + 16 * kk, 32 * ib);
    } else {
      const int h = lane_id() >> 5;
      return grow[(size_t)sfeat(t, kk, h) * W + 32 * ib + (lane_id() & 31)];
    }
  }
};

// One output block of a layer: sum over input blocks and k-steps.
template <int PREC, int NIB, class AF>
__device__ __forceinline__ floatx16 layer_block(const AF& af, int ob, const uint32_t (&X)[NIB][PR<PREC>::SR]) {
  using P = PR<PREC>;
  floatx16 acc = {};
#pragma unroll
  for (int t = 0; t < NIB; ++t)
#pragma unroll
    for (int kk = 0; kk < P::KS; ++kk) acc = P::mma(af(ob, t, kk), P::sfrag(X[t], kk), acc);
  return acc;
}

__device__ __forceinline__ void bias_relu(floatx16& a, const float* bias, int ob) {
  const int h = lane_id() >> 5;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    float v = a[r] + bias[sfeat(ob, r, h)];
    a[r] = v > 0.f ? v : 0.f;
  }
}

// Loss value and dL/dy of one sample (batch-mean losses).
template <int C>
__device__ __forceinline__ float loss_grad(const SampleSpec& sp, const Smp& s, int64_t j, const float (&y)[C],
                                           float (&gy)[C]) {
  float L = 0.f;
  if (!s.valid) {
#pragma unroll
    for (int c = 0; c < C; ++c) gy[c] = 0.f;
    return 0.f;
  }
  if (sp.loss == LOSS_EXTERNAL) {
#pragma unroll
    for (int c = 0; c < C; ++c) gy[c] = sp.gy[(size_t)j * C + c];
    return 0.f;
  }
  if constexpr (C == 1) {
    if (sp.loss == LOSS_MSE) {
      float d = y[0] - s.t;
      L = d * d;
      gy[0] = 2.f * d * sp.inv_n;
    } else {  // BCE on a logit
      float e = __expf(-fabsf(y[0]));
      L = fmaxf(y[0], 0.f) - y[0] * s.t + log1pf(e);
      float sig = y[0] >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
      gy[0] = (sig - s.t) * sp.inv_n;
    }
  } else {  // CE over C logits
    float mx = y[0];
#pragma unroll
    for (int c = 1; c < C; ++c) mx = fmaxf(mx, y[c]);
    float se = 0.f, e[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      e[c] = __expf(y[c] - mx);
      se += e[c];
    }
    float yc = y[0];
#pragma unroll
    for (int c = 1; c < C; ++c) yc = (s.cls == c) ? y[c] : yc;
    L = mx + __logf(se) - yc;
#pragma unroll
    for (int c = 0; c < C; ++c) gy[c] = (e[c] / se - (s.cls == c ? 1.f : 0.f)) * sp.inv_n;
  }
  return L;
}

// ============================================================== training kernel
template <int PREC, int W, int H, int KP, int C>
struct TrainCfg {
  static constexpr int NB = W / 32, NIB0 = KP / 32, NSLOT = 2;
  // Layers whose dW stays in registers for the whole step (BF16 form); the others
  // fold each iteration's contribution into the work-group's partial row in HBM.
  static constexpr bool DWREG = (PREC == NVDB_BF16);
  static constexpr int DWREG_FROM = (W >= 128) ? 1 : 0;
  static constexpr bool reg_layer(int l) { return DWREG && l >= DWREG_FROM; }
  static constexpr bool any_rmw = !DWREG || DWREG_FROM > 0;
  static constexpr int FPW = W / 4;                   // bias/head features owned per wave
  static constexpr int RB = (PREC == NVDB_BF16) ? 0 : (KP > W ? KP : W) + 4;  // fp32 row pitch (floats)
  static constexpr int ROWS_BYTES = (PREC == NVDB_BF16) ? 32 * ROW_ELEMS * 2 : 32 * RB * 4;
  static constexpr int SLOT_BYTES = 2 * ROWS_BYTES + 32 * C * 4;
  static constexpr int WL_BYTES = (PREC == NVDB_BF16) ? (H - 1) * W * ROW_ELEMS * 2 : 0;
  static constexpr int SMALL_FLOATS = H * W + C * W + 4 + 3 * (KP / 2) + 8;
  static constexpr int LDS_BYTES = WL_BYTES + NSLOT * SLOT_BYTES + SMALL_FLOATS * 4;
  // dW blocks owned by a wave: waves form a 2 x 2 grid over (output, input) blocks.
  static constexpr int OBW = NB / 2;
  static constexpr int IBW0 = NIB0 / 2, IBW = NB / 2;
  static constexpr int IBWMAX = IBW0 > IBW ? IBW0 : IBW;
};


template <int PREC, int W, int H, int KP, int C>
__global__ void __launch_bounds__(256, 1) __attribute__((amdgpu_waves_per_eu(1, 1))) k_train(TrainLaunch L) {
  using P = PR<PREC>;
  using CF = TrainCfg<PREC, W, H, KP, C>;
  constexpr int NB = CF::NB, NIB0 = CF::NIB0, SR = P::SR, OBW = CF::OBW, FPW = CF::FPW;
  constexpr bool BF = (PREC == NVDB_BF16);
  __shared__ __attribute__((aligned(16))) char smem[CF::LDS_BYTES];

  const TrainNet& TN = L.nets[blockIdx.y];
  const NetView& nv = TN.net;
  const SampleSpec& sp = TN.spec;
  const int lane = lane_id(), wave = wave_id(), h = lane >> 5, fl = lane & 31;
  const int64_t P_ = nv.s.nparams();

  // ---- LDS carve-up
  __bf16* wl0 = (__bf16*)smem;                                   // bf16 layers 1..H-1
  char* slots = smem + CF::WL_BYTES;
  float* sm_bias0 = (float*)(slots + CF::NSLOT * CF::SLOT_BYTES);  // [H][W]
  float* sm_whead0 = sm_bias0 + H * W;                             // [C][W]
  float* sm_bhead0 = sm_whead0 + C * W;                            // [C] (padded to 4)
  float* sm_benc0 = sm_bhead0 + 4;                                 // [KP/2][3]
  float* sm_red = sm_benc0 + 3 * (KP / 2);                         // [8] reductions

  // ---- stage parameters
  if constexpr (BF) {
    const u32x4* src = (const u32x4*)((const __bf16*)nv.wrow + (size_t)W * ROW_ELEMS);  // skip layer 0
    u32x4* dst = (u32x4*)wl0;
    for (int i = threadIdx.x; i < CF::WL_BYTES / 16; i += blockDim.x) dst[i] = src[i];
  }
  for (int i = threadIdx.x; i < H * W; i += blockDim.x) sm_bias0[i] = nv.bias[i];
  for (int i = threadIdx.x; i < C * W; i += blockDim.x) sm_whead0[i] = nv.whead[i];
  if (threadIdx.x < C) sm_bhead0[threadIdx.x] = nv.bhead[threadIdx.x];
  for (int i = threadIdx.x; i < 3 * (KP / 2); i += blockDim.x) sm_benc0[i] = nv.benc[i];
  __syncthreads();

  // ---- per-wave accumulators kept across iterations
  floatx16 dacc[H][OBW][CF::IBWMAX];
#pragma unroll
  for (int l = 0; l < H; ++l)
#pragma unroll
    for (int a = 0; a < OBW; ++a)
#pragma unroll
      for (int b = 0; b < CF::IBWMAX; ++b) dacc[l][a][b] = floatx16{};
  float dbias[H];
#pragma unroll
  for (int l = 0; l < H; ++l) dbias[l] = 0.f;
  float dwh[C], dbh[C];
#pragma unroll
  for (int c = 0; c < C; ++c) dwh[c] = dbh[c] = 0.f;
  float loss_acc = 0.f;

  const int wo = wave >> 1, wi = wave & 1;
  const int64_t n_iter = (sp.n + 127) / 128;
  float* partial = TN.partial + (size_t)blockIdx.x * P_;


  for (int64_t it = blockIdx.x; it < n_iter; it += L.G) {
    const int z = opaque_zero();
    const float* sm_bias = sm_bias0 + z;
    const float* sm_whead = sm_whead0 + z;
    const float* sm_bhead = sm_bhead0 + z;
    const float* sm_benc = sm_benc0 + z;
    __bf16* wl = wl0 + z;
    const int64_t j = it * 128 + wave * 32 + fl;
    const Smp smp = fetch_sample(sp, L.tree, j);

    // ================= forward
    uint32_t Hs[H][NB][SR];  // Hs[l] = a_{l+1} (S layout), l = 0..H-1
    {
      WFwd<PREC, W, KP> wf0{nullptr, (const u32x4*)nv.w1frag + z, (const float*)nv.wcol + z, 0};
      uint32_t X0[NIB0][SR];
      encode_S<PREC, NIB0>(smp, sm_benc, nv.nfreq, X0);
#pragma unroll
      for (int ob = 0; ob < NB; ++ob) {
        floatx16 a = layer_block<PREC, NIB0>(wf0, ob, X0);
        bias_relu(a, sm_bias, ob);
        P::store(a, Hs[0][ob]);
      }
    }
    static_for<1, H>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      WFwd<PREC, W, KP> wf{wl + (size_t)(l - 1) * W * ROW_ELEMS, nullptr,
                           (const float*)nv.wcol + z + (size_t)KP * W + (size_t)(l - 1) * W * W, l};
#pragma unroll
      for (int ob = 0; ob < NB; ++ob) {
        floatx16 a = layer_block<PREC, NB>(wf, ob, Hs[l - 1]);
        bias_relu(a, sm_bias + l * W, ob);
        P::store(a, Hs[l][ob]);
      }
    });
    // head (VALU): y_c = sum_f Wh[c][f] a_H[f] + bh[c]
    float y[C], gy[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      float acc = 0.f;
#pragma unroll
      for (int ob = 0; ob < NB; ++ob)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          float av;
          if constexpr (BF) {
            uint32_t w = Hs[H - 1][ob][r >> 1];
            av = __uint_as_float((r & 1) ? (w & 0xffff0000u) : (w << 16));
          } else {
            av = __uint_as_float(Hs[H - 1][ob][r]);
          }
          acc = fmaf(sm_whead[c * W + sfeat(ob, r, h)], av, acc);
        }
      y[c] = acc + shfl_xor32(acc) + sm_bhead[c];
    }
    const float Ls = loss_grad<C>(sp, smp, j, y, gy);
    if (h == 0) loss_acc += Ls;

    // g_H = (Wh^T gy) * 1[a_H > 0]
    uint32_t Gc[NB][SR];
#pragma unroll
    for (int ob = 0; ob < NB; ++ob) {
      floatx16 g;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        float v = 0.f;
#pragma unroll
        for (int c = 0; c < C; ++c) v = fmaf(sm_whead[c * W + sfeat(ob, r, h)], gy[c], v);
        g[r] = P::positive(Hs[H - 1][ob], r) ? v : 0.f;
      }
      P::store(g, Gc[ob]);
    }

    // ================= head gradients (rows of a_H and gy exchanged through LDS)
#pragma unroll
    for (int round = 0; round < 4 / CF::NSLOT; ++round) {
      const int my_slot = wave - round * CF::NSLOT;
      if (my_slot >= 0 && my_slot < CF::NSLOT) {
        char* sl = slots + my_slot * CF::SLOT_BYTES;
        if constexpr (BF) write_rows_bf16<NB>((__bf16*)(sl + CF::ROWS_BYTES), Hs[H - 1]);
        else write_rows_f32<NB>((float*)(sl + CF::ROWS_BYTES), CF::RB, Hs[H - 1]);
        if (h == 0) {
          float* gyr = (float*)(sl + 2 * CF::ROWS_BYTES);
#pragma unroll
          for (int c = 0; c < C; ++c) gyr[fl * C + c] = gy[c];
        }
      }
      __syncthreads();
#pragma unroll
      for (int sl_i = 0; sl_i < CF::NSLOT; ++sl_i) {
        const char* sl = slots + sl_i * CF::SLOT_BYTES;
        const float* gyr = (const float*)(sl + 2 * CF::ROWS_BYTES);
        if (fl < FPW) {
          const int f = FPW * wave + fl;
#pragma unroll 4
          for (int s = h; s < 32; s += 2) {
            float av;
            if constexpr (BF) av = row_elem_bf16((const __bf16*)(sl + CF::ROWS_BYTES), s, f);
            else av = ((const float*)(sl + CF::ROWS_BYTES))[s * CF::RB + f];
#pragma unroll
            for (int c = 0; c < C; ++c) dwh[c] = fmaf(gyr[s * C + c], av, dwh[c]);
          }
        }
        if (wave == 0) {
#pragma unroll
          for (int c = 0; c < C; ++c) {
            if (fl == c) {
              float acc = 0.f;
              for (int s = h; s < 32; s += 2) acc += gyr[s * C + c];
              dbh[c] += acc;
            }
          }
        }
      }
      __syncthreads();
    }

    // ================= backward through the hidden layers
    static_for<0, H>([&](auto kc) {
      constexpr int l = H - 1 - decltype(kc)::value;
      constexpr int NIBl = (l == 0) ? NIB0 : NB;
      constexpr int IBWl = NIBl / 2;
      // input activations a_l of layer l as rows (gamma recomputed for l = 0)
      uint32_t X0[NIB0][SR];
      if constexpr (l == 0) encode_S<PREC, NIB0>(smp, sm_benc, nv.nfreq, X0);

#pragma unroll
      for (int round = 0; round < 4 / CF::NSLOT; ++round) {
        const int my_slot = wave - round * CF::NSLOT;
        if (my_slot >= 0 && my_slot < CF::NSLOT) {
          char* sl = slots + my_slot * CF::SLOT_BYTES;
          if constexpr (BF) {
            write_rows_bf16<NB>((__bf16*)sl, Gc);
            if constexpr (l == 0) write_rows_bf16<NIB0>((__bf16*)(sl + CF::ROWS_BYTES), X0);
            else write_rows_bf16<NB>((__bf16*)(sl + CF::ROWS_BYTES), Hs[l - 1 < 0 ? 0 : l - 1]);
          } else {
            write_rows_f32<NB>((float*)sl, CF::RB, Gc);
            if constexpr (l == 0) write_rows_f32<NIB0>((float*)(sl + CF::ROWS_BYTES), CF::RB, X0);
            else write_rows_f32<NB>((float*)(sl + CF::ROWS_BYTES), CF::RB, Hs[l - 1 < 0 ? 0 : l - 1]);
          }
        }
        __syncthreads();
#pragma unroll
        for (int sl_i = 0; sl_i < CF::NSLOT; ++sl_i) {
          const char* sl = slots + sl_i * CF::SLOT_BYTES;
#pragma unroll
          for (int kk = 0; kk < P::KS; ++kk) {
            typename P::Frag ga[OBW], hb[CF::IBWMAX];
#pragma unroll
            for (int a = 0; a < OBW; ++a) {
              const int ob = wo * OBW + a;
              if constexpr (BF) ga[a] = frag_cols_bf16((const __bf16*)sl, 16 * kk, 32 * ob);
              else ga[a] = ((const float*)sl)[(2 * kk + h) * CF::RB + 32 * ob + fl];
            }
#pragma unroll
            for (int b = 0; b < CF::IBWMAX; ++b) {
              if (b < IBWl) {
                const int ib = wi * IBWl + b;
                if constexpr (BF) hb[b] = frag_cols_bf16((const __bf16*)(sl + CF::ROWS_BYTES), 16 * kk, 32 * ib);
                else hb[b] = ((const float*)(sl + CF::ROWS_BYTES))[(2 * kk + h) * CF::RB + 32 * ib + fl];
              }
            }
#pragma unroll
            for (int a = 0; a < OBW; ++a)
#pragma unroll
              for (int b = 0; b < CF::IBWMAX; ++b)
                if (b < IBWl) dacc[l][a][b] = P::mma(ga[a], hb[b], dacc[l][a][b]);
          }
          // bias gradient: column sums of the g rows
          if (fl < FPW) {
            const int f = FPW * wave + fl;
            float acc = 0.f;
#pragma unroll 4
            for (int s = h; s < 32; s += 2) {
              if constexpr (BF) acc += row_elem_bf16((const __bf16*)sl, s, f);
              else acc += ((const float*)sl)[s * CF::RB + f];
            }
            dbias[l] += acc;
          }
        }
        __syncthreads();
      }

      if constexpr (!CF::reg_layer(l)) {
        // fold this iteration's blocks into the work-group's partial row
#pragma unroll
        for (int a = 0; a < OBW; ++a)
#pragma unroll
          for (int b = 0; b < CF::IBWMAX; ++b) {
            if (b < IBWl) {
              const int ob = wo * OBW + a, ib = wi * IBWl + b;
              const int win = nv.s.win(l);
              const int i = 32 * ib + fl;
              if (i < win) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                  const int o = sfeat(ob, r, h);
                  float* p = partial + nv.s.woff(l) + (size_t)o * win + i;
                  *p += dacc[l][a][b][r];
                }
              }
              dacc[l][a][b] = floatx16{};
            }
          }
      }

      if constexpr (l > 0) {
        // g_l = (W_l^T g_{l+1}) * 1[a_l > 0]
        WBwd<PREC, W> wb{wl + (size_t)(l - 1) * W * ROW_ELEMS,
                         (const float*)nv.wrow + z + (size_t)W * KP + (size_t)(l - 1) * W * W};
        uint32_t Gn[NB][SR];
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) {
          floatx16 a = layer_block<PREC, NB>(wb, ib, Gc);
#pragma unroll
          for (int r = 0; r < 16; ++r) a[r] = P::positive(Hs[l - 1][ib], r) ? a[r] : 0.f;
          P::store(a, Gn[ib]);
        }
#pragma unroll
        for (int ib = 0; ib < NB; ++ib)
#pragma unroll
          for (int q = 0; q < SR; ++q) Gc[ib][q] = Gn[ib][q];
      }
    });
  }

  // ---- write this work-group's partial gradient row
  if constexpr (CF::DWREG) {
    static_for<0, H>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      if constexpr (!CF::reg_layer(l)) return;
      constexpr int NIBl = (l == 0) ? NIB0 : NB;
      constexpr int IBWl = NIBl / 2;
      const int win = nv.s.win(l);
#pragma unroll
      for (int a = 0; a < OBW; ++a)
#pragma unroll
        for (int b = 0; b < CF::IBWMAX; ++b) {
          if (b < IBWl) {
            const int ob = wo * OBW + a, ib = wi * IBWl + b;
            const int i = 32 * ib + fl;
            if (i < win) {
#pragma unroll
              for (int r = 0; r < 16; ++r) {
                const int o = sfeat(ob, r, h);
                partial[nv.s.woff(l) + (size_t)o * win + i] = dacc[l][a][b][r];
              }
            }
          }
        }
    });
  }
  // biases and head: combine the two lane halves, lanes of the low half write
#pragma unroll
  for (int l = 0; l < H; ++l) {
    float v = dbias[l] + shfl_xor32(dbias[l]);
    if (h == 0 && fl < FPW) partial[nv.s.boff(l) + FPW * wave + fl] = v;
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    float v = dwh[c] + shfl_xor32(dwh[c]);
    if (h == 0 && fl < FPW) partial[nv.s.woff(H) + (size_t)c * W + FPW * wave + fl] = v;
    float b = dbh[c] + shfl_xor32(dbh[c]);
    if (wave == 0 && h == 0 && fl == c) partial[nv.s.boff(H) + c] = b;
  }
  // loss: fixed-order reduction over the wave, then over the four waves
  float v = loss_acc;
#pragma unroll
  for (int off = 16; off >= 1; off >>= 1) {
    int src = (lane ^ off) << 2;
    v += __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v)));
  }
  if (lane == 0) sm_red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) TN.loss_partial[blockIdx.x] = ((sm_red[0] + sm_red[1]) + sm_red[2]) + sm_red[3];
}

// ============================================================== inference kernel

template <int PREC, int W, int H, int KP, int C>
struct InferCfg {
  static constexpr int NT = (PREC == NVDB_BF16) ? 2 : 1;  // 32-sample tiles per wave sharing each weight fragment
  static constexpr int WL_BYTES = (PREC == NVDB_BF16) ? H * W * ROW_ELEMS * 2 : 0;
  static constexpr int SMALL_FLOATS = H * W + C * W + 4 + 3 * (KP / 2);
  static constexpr int LDS_BYTES = WL_BYTES + SMALL_FLOATS * 4;
};

template <int PREC, int W, int H, int KP, int C>
__global__ void __launch_bounds__(256, 1) __attribute__((amdgpu_waves_per_eu(1, 1))) k_infer(InferLaunch I) {
  using P = PR<PREC>;
  using CF = InferCfg<PREC, W, H, KP, C>;
  constexpr int NB = W / 32, NIB0 = KP / 32, SR = P::SR, NT = CF::NT;
  constexpr bool BF = (PREC == NVDB_BF16);
  __shared__ __attribute__((aligned(16))) char smem[CF::LDS_BYTES];
  const NetView& nv = I.net;
  const SampleSpec& sp = I.spec;
  const int lane = lane_id(), wave = wave_id(), h = lane >> 5, fl = lane & 31;

  __bf16* wl0 = (__bf16*)smem;
  float* sm_bias0 = (float*)(smem + CF::WL_BYTES);
  float* sm_whead0 = sm_bias0 + H * W;
  float* sm_bhead0 = sm_whead0 + C * W;
  float* sm_benc0 = sm_bhead0 + 4;
  if constexpr (BF) {
    const u32x4* src = (const u32x4*)nv.wrow;
    u32x4* dst = (u32x4*)wl0;
    for (int i = threadIdx.x; i < CF::WL_BYTES / 16; i += blockDim.x) dst[i] = src[i];
  }
  for (int i = threadIdx.x; i < H * W; i += blockDim.x) sm_bias0[i] = nv.bias[i];
  for (int i = threadIdx.x; i < C * W; i += blockDim.x) sm_whead0[i] = nv.whead[i];
  if (threadIdx.x < C) sm_bhead0[threadIdx.x] = nv.bhead[threadIdx.x];
  for (int i = threadIdx.x; i < 3 * (KP / 2); i += blockDim.x) sm_benc0[i] = nv.benc[i];
  __syncthreads();

  const int64_t per_wave = 32 * NT;
  const int64_t stride = (int64_t)gridDim.x * 4 * per_wave;
  for (int64_t base = ((int64_t)blockIdx.x * 4 + wave) * per_wave; base < sp.n; base += stride) {
    const int z = opaque_zero();
    const float* sm_bias = sm_bias0 + z;
    const float* sm_whead = sm_whead0 + z;
    const float* sm_bhead = sm_bhead0 + z;
    const float* sm_benc = sm_benc0 + z;
    __bf16* wl = wl0 + z;
    uint32_t A[NT][NB > NIB0 ? NB : NIB0][SR];
    Smp smp[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      smp[u] = fetch_sample(sp, I.tree, base + 32 * u + fl);
      uint32_t X0[NIB0][SR];
      encode_S<PREC, NIB0>(smp[u], sm_benc, nv.nfreq, X0);
#pragma unroll
      for (int t = 0; t < NIB0; ++t)
#pragma unroll
        for (int q = 0; q < SR; ++q) A[u][t][q] = X0[t][q];
    }
    static_for<0, H>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      constexpr int NIBl = (l == 0) ? NIB0 : NB;
      WFwd<PREC, W, KP> wf{wl + (size_t)l * W * ROW_ELEMS, (const u32x4*)nv.w1frag + z,
                           (const float*)nv.wcol + z + (l == 0 ? 0 : (size_t)KP * W + (size_t)(l - 1) * W * W), BF ? 1 : l};
      uint32_t Bn[NT][NB][SR];
#pragma unroll
      for (int ob = 0; ob < NB; ++ob) {
        floatx16 acc[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u) acc[u] = floatx16{};
#pragma unroll
        for (int t = 0; t < (NB > NIB0 ? NB : NIB0); ++t) {
          if (t < NIBl) {
#pragma unroll
            for (int kk = 0; kk < P::KS; ++kk) {
              typename P::Frag af = wf(ob, t, kk);
#pragma unroll
              for (int u = 0; u < NT; ++u) acc[u] = P::mma(af, P::sfrag(A[u][t], kk), acc[u]);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          bias_relu(acc[u], sm_bias + l * W, ob);
          P::store(acc[u], Bn[u][ob]);
        }
      }
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int t = 0; t < NB; ++t)
#pragma unroll
          for (int q = 0; q < SR; ++q) A[u][t][q] = Bn[u][t][q];
    });
    // head
    float y[NT][C];
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        float acc = 0.f;
#pragma unroll
        for (int ob = 0; ob < NB; ++ob)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            float av;
            if constexpr (BF) {
              uint32_t w = A[u][ob][r >> 1];
              av = __uint_as_float((r & 1) ? (w & 0xffff0000u) : (w << 16));
            } else {
              av = __uint_as_float(A[u][ob][r]);
            }
            acc = fmaf(sm_whead[c * W + sfeat(ob, r, h)], av, acc);
          }
        y[u][c] = acc + shfl_xor32(acc) + sm_bhead[c];
      }
    // outputs
    if (I.out_kind == OUT_MASK) {
      uint64_t b0 = __ballot(y[0][0] > 0.f) & 0xffffffffull;
      uint64_t b1 = __ballot((NT > 1 ? y[NT - 1][0] : 0.f) > 0.f) & 0xffffffffull;
      if (lane == 0 && base < sp.n) I.mask[base >> 6] = b0 | (b1 << 32);
    } else {
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const int64_t j = base + 32 * u + fl;
        if (h == 0 && j < sp.n) {
          if (I.out_kind == OUT_VALUES) {
            I.y[j] = y[u][0] * I.out_scale;
          } else if (I.out_kind == OUT_CLASS) {
            int best = 0;
            float bv = y[u][0];
#pragma unroll
            for (int c = 1; c < C; ++c)
              if (y[u][c] > bv) { bv = y[u][c]; best = c; }
            I.cls[j] = (uint8_t)best;
          } else {
#pragma unroll
            for (int c = 0; c < C; ++c) I.y[(size_t)j * C + c] = y[u][c];
          }
        }
      }
    }
  }
}

// ============================================================== reduce + Adam

__device__ __forceinline__ void write_shadow(const AdamNet& A, int64_t p, float th) {
  const NetShape& s = A.s;
  int l = 0;
  while (l < s.H && p >= s.woff(l + 1)) ++l;
  const int64_t wend = s.boff(l);
  if (l == s.H) {  // head
    if (p < wend) A.whead[p - s.woff(l)] = th;
    else A.bhead[p - wend] = th;
    return;
  }
  if (p >= wend) {
    A.bias[l * s.W + (p - wend)] = th;
    return;
  }
  const int win = s.win(l);
  const int o = (int)((p - s.woff(l)) / win), i = (int)((p - s.woff(l)) % win);
  if (A.prec == NVDB_BF16) {
    __bf16* rows = (__bf16*)A.wrow + (size_t)l * s.W * ROW_ELEMS;
    rows[(size_t)o * ROW_ELEMS + swz_elem(o, i)] = (__bf16)th;
    if (l == 0) {
      const int ob = o >> 5, ii = o & 31, t = i >> 5, rem = i & 31, kk = rem >> 4, rr = rem & 15;
      const int e = ((rr >> 3) << 2) | (rr & 3), hh = (rr >> 2) & 1;
      const int lane = ii + 32 * hh;
      ((__bf16*)A.w1frag)[((((size_t)ob * (s.KP / 32) + t) * 2 + kk) * 64 + lane) * 8 + e] = (__bf16)th;
    }
  } else {
    const size_t loff = (l == 0) ? 0 : (size_t)s.KP * s.W + (size_t)(l - 1) * s.W * s.W;
    ((float*)A.wrow)[loff + (size_t)o * (l == 0 ? s.KP : s.W) + i] = th;
    ((float*)A.wcol)[loff + (size_t)i * s.W + o] = th;
  }
}

__global__ void __launch_bounds__(256) k_reduce_adam(AdamLaunch AL) {
  const AdamNet& A = AL.nets[blockIdx.y];
  const int64_t P = A.s.nparams();
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0 && A.loss_out) {
    float L = 0.f;
    for (int g = 0; g < A.G; ++g) L += A.loss_partial[g];
    *A.loss_out = L * A.loss_scale;
  }
  if (p >= P) return;
  float g = 0.f;
  for (int w = 0; w < A.G; ++w) g += A.partial[(size_t)w * P + p];
  if (A.grad_out) {
    A.grad_out[p] = g;
    return;
  }
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float m = b1 * A.m[p] + (1.f - b1) * g;
  float v = b2 * A.v[p] + (1.f - b2) * g * g;
  A.m[p] = m;
  A.v[p] = v;
  float th = A.theta[p] - A.lr * (m / A.bc1) / (sqrtf(v / A.bc2) + eps);
  A.theta[p] = th;
  write_shadow(A, p, th);
}

// Rebuild every shadow copy from the master parameters (after set_params).
__global__ void k_write_shadow(AdamNet A) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < A.s.nparams()) write_shadow(A, p, A.theta[p]);
}

__global__ void k_sample(uint64_t sseed, uint32_t npop, int64_t n, uint32_t* out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = (uint32_t)__umul64hi(sm_mix(sseed + SM_GOLDEN * (uint64_t)(j + 1)), (uint64_t)npop);
}

// ============================================================== host dispatch

template <int PREC, int W, int H, int KP, int C>
KernelSet make_set() {
  return KernelSet{k_train<PREC, W, H, KP, C>, k_infer<PREC, W, H, KP, C>,
                   TrainCfg<PREC, W, H, KP, C>::LDS_BYTES, InferCfg<PREC, W, H, KP, C>::LDS_BYTES,
                   TrainCfg<PREC, W, H, KP, C>::any_rmw};
}

// Shapes with compiled kernels: (W, H, KP, C).
#define NVDB_FOR_SHAPES(X) \
  X(64, 3, 64, 1)          \
  X(64, 4, 128, 3)         \
  X(128, 4, 128, 1)        \
  X(128, 3, 128, 1)

bool find_kernels(int prec, int W, int H, int KP, int C, KernelSet* out) {
#define NVDB_MATCH(w, hh, kp, c)                                                      \
  if (W == w && H == hh && KP == kp && C == c) {                                      \
    *out = prec == NVDB_BF16 ? make_set<NVDB_BF16, w, hh, kp, c>() : make_set<NVDB_FP32, w, hh, kp, c>(); \
    return true;                                                                      \
  }
  NVDB_FOR_SHAPES(NVDB_MATCH)
#undef NVDB_MATCH
  return false;
}

void launch_train(const KernelSet& ks, const TrainLaunch& L, int n_nets, hipStream_t st) {
  hipLaunchKernelGGL(ks.train, dim3(L.G, n_nets), dim3(256), 0, st, L);
  NVDB_HIP(hipGetLastError());
}
void launch_infer(const KernelSet& ks, const InferLaunch& I, int grid, hipStream_t st) {
  hipLaunchKernelGGL(ks.infer, dim3(grid), dim3(256), 0, st, I);
  NVDB_HIP(hipGetLastError());
}
void launch_reduce_adam(const AdamLaunch& A, int64_t max_p, int n_nets, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_adam, dim3((unsigned)((max_p + 255) / 256), n_nets), dim3(256), 0, st, A);
  NVDB_HIP(hipGetLastError());
}
void launch_write_shadow(const AdamNet& A, hipStream_t st) {
  hipLaunchKernelGGL(k_write_shadow, dim3((unsigned)((A.s.nparams() + 255) / 256)), dim3(256), 0, st, A);
  NVDB_HIP(hipGetLastError());
}
void launch_sample(uint64_t sseed, uint32_t npop, int64_t n, uint32_t* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_sample, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sseed, npop, n, out);
  NVDB_HIP(hipGetLastError());
}

}  // namespace nvdb
