// Device-side building blocks of the coordinate-MLP kernels (gfx950), shared by
// the translation units of the training and inference kernels: lane layout,
// sample fetch and draw, the feature mapping, LDS row layout, weight fragments,
// layer products and losses.  Everything here is inline.
#pragma once
#include "nvdb_internal.h"


namespace nvdb {

// Launch and pipeline constants, each chosen by measurement on the 512^3 level-set
// workload.  Decode: eight waves per work-group (two per SIMD) share one LDS copy of
// the weights, so one wave's conversions overlap the other's matrix products, each
// wave two 32-sample tiles.  FP8 decode: the e4m3 weights take 64 KiB of LDS, so two
// work-groups of eight single-tile waves fit on a CU (four waves per SIMD).
// Activation-rows training kernel: forward weight fragments 4 steps ahead, input-
// gradient fragments 2 steps ahead (deeper prefetch spills registers and is slower).
constexpr int INFER_WAVES = 8;
constexpr int INFER_NT = 2;
constexpr int INFER8_WAVES = 8;
constexpr int INFER8_NT = 1;
constexpr int INFER8_WGS = 2;
constexpr int ROWS_FWD_PF = 4;
constexpr int ROWS_DX_PF = 2;



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
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
// Two floats to packed bf16 (round to nearest even), a in the low half.  A vector
// conversion becomes one two-source instruction; converting the values one at a
// time costs two conversions and a permute.
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  const floatx2 f = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2));
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

typedef short short2v __attribute__((ext_vector_type(2)));
typedef unsigned short ushort2v __attribute__((ext_vector_type(2)));
// ReLU of two packed bf16 values: read as int16, negative bf16 values are negative.
__device__ __forceinline__ uint32_t relu_pk(uint32_t w) {
  short2v v = __builtin_bit_cast(short2v, w);
  v = __builtin_elementwise_max(v, short2v{0, 0});
  return __builtin_bit_cast(uint32_t, v);
}
// Zero the halves of the 8 words g whose matching half of a (a ReLU output, so
// >= +0) is zero: t = min(a, 1) per 16-bit half is 1 where a > 0 and 0 where
// a == 0, and the 16-bit product g * t keeps or clears each half.  The products
// are inline assembly because the optimiser turns a product by {0, 1}, and the
// minimum too, into per-half compares and selects.  The compiler does not count inline assembly as
// a vector-ALU write when it pads matrix-core operand reads, so one trailing s_nop
// supplies the two wait states a matrix product reading the last word right away
// would need (the earlier words are followed by the later products).
__device__ __forceinline__ void mask_pk8(uint32_t (&g)[8], const uint32_t* a) {
  uint32_t t[8];
  asm("v_pk_min_u16 %8, %16, %24\n\t"
      "v_pk_min_u16 %9, %17, %24\n\t"
      "v_pk_min_u16 %10, %18, %24\n\t"
      "v_pk_min_u16 %11, %19, %24\n\t"
      "v_pk_min_u16 %12, %20, %24\n\t"
      "v_pk_min_u16 %13, %21, %24\n\t"
      "v_pk_min_u16 %14, %22, %24\n\t"
      "v_pk_min_u16 %15, %23, %24\n\t"
      "v_pk_mul_lo_u16 %0, %0, %8\n\t"
      "v_pk_mul_lo_u16 %1, %1, %9\n\t"
      "v_pk_mul_lo_u16 %2, %2, %10\n\t"
      "v_pk_mul_lo_u16 %3, %3, %11\n\t"
      "v_pk_mul_lo_u16 %4, %4, %12\n\t"
      "v_pk_mul_lo_u16 %5, %5, %13\n\t"
      "v_pk_mul_lo_u16 %6, %6, %14\n\t"
      "v_pk_mul_lo_u16 %7, %7, %15\n\t"
      "s_nop 1"
      : "+v"(g[0]), "+v"(g[1]), "+v"(g[2]), "+v"(g[3]), "+v"(g[4]), "+v"(g[5]), "+v"(g[6]), "+v"(g[7]),
        "=&v"(t[0]), "=&v"(t[1]), "=&v"(t[2]), "=&v"(t[3]), "=&v"(t[4]), "=&v"(t[5]), "=&v"(t[6]), "=&v"(t[7])
      : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5]), "v"(a[6]), "v"(a[7]), "s"(0x00010001u));
}
template <int PREC>
__device__ __forceinline__ void store_relu(floatx16 a, uint32_t* s) {
  if constexpr (PREC == NVDB_BF16) {
    PR<PREC>::store(a, s);
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] = relu_pk(s[i]);
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i) s[i] = __float_as_uint(a[i] > 0.f ? a[i] : 0.f);
  }
}
// Store a gradient block masked by the ReLU derivative of the activation block act.
template <int PREC>
__device__ __forceinline__ void store_masked(floatx16 a, uint32_t* s, const uint32_t* act) {
  if constexpr (PREC == NVDB_BF16) {
    uint32_t w[8];
    PR<PREC>::store(a, w);
    mask_pk8(w, act);
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] = w[i];
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i) s[i] = __uint_as_float(act[i]) > 0.f ? __float_as_uint(a[i]) : 0u;
  }
}

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

// `count` selects the one caller per sample that counts an out-of-range index (the two
// lane halves of a decode wave fetch the same sample).
__device__ __forceinline__ Smp fetch_sample(const SampleSpec& sp, const TreeView& tv, int64_t j, bool count = true) {
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
    if (g >= sp.npop) {  // out of the population: read index 0 and count it
      if (sp.bad_idx && count) atomicAdd(sp.bad_idx, 1ull);
      g = 0;
    }
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
    if (!sp.direct) s.t = tv.values[g] * sp.tscale;  // decoding needs no target
  } else if (sp.src == SRC_LEAF_SLOTS) {
    uint32_t leaf = g >> 9, n0 = g & 511u;
    int4 o = tv.leaf_o[leaf];
    px = o.x + (int)(n0 >> 6);
    py = o.y + (int)((n0 >> 3) & 7u);
    pz = o.z + (int)(n0 & 7u);
    if (!sp.direct) s.t = (float)((tv.leaf_mask[(size_t)leaf * 8 + (n0 >> 6)] >> (n0 & 63u)) & 1ull);
  } else {  // SRC_L1_SLOTS (every slot of the level-1 nodes) or SRC_TILES: leaf centres
    const bool tile = sp.src == SRC_TILES;
    const uint32_t key = tile ? tv.tile_key[g] : g;
    uint32_t node = key >> 12, n1 = key & 4095u;
    int4 o = tv.l1_o[node];
    px = o.x + 8 * (int)(n1 >> 8);
    py = o.y + 8 * (int)((n1 >> 4) & 15u);
    pz = o.z + 8 * (int)(n1 & 15u);
    half = 4.f;
    if (!sp.direct) {
      if (tile) {
        s.t = tv.tile_val[g] * sp.tscale;
      } else {
        const uint64_t c = (tv.l1_child[(size_t)node * 64 + (n1 >> 6)] >> (n1 & 63u)) & 1ull;
        const uint64_t a = (tv.l1_active[(size_t)node * 64 + (n1 >> 6)] >> (n1 & 63u)) & 1ull;
        s.cls = c ? 0 : (a ? 1 : 2);
      }
    }
  }
  s.x[0] = ((float)(px - sp.lo[0]) + half) * sp.inv_d;
  s.x[1] = ((float)(py - sp.lo[1]) + half) * sp.inv_d;
  s.x[2] = ((float)(pz - sp.lo[2]) + half) * sp.inv_d;
  return s;
}

// The next tile's sample of a training lane, fetched while the current tile runs.
// With the i.i.d. sampler over active voxels or leaf slots the kernel draws it
// itself (the arithmetic of fetch_sample, split so that no load result is used in
// the stage that issues it): stage 1 forms the population index and loads the
// voxel key and value (voxels) or the leaf origin and mask word (leaf slots);
// stage 2, later in the tile, loads a voxel's leaf origin.  Otherwise stage 1
// reads the gathered record (x, y, z, target or class) into o.  Only the BF16
// kernels draw their own samples (FUSE); in the FP32 form the registers are scarcer.
struct NextSample {
  uint32_t key;  // voxel key, or population index of a leaf slot
  uint2 aux;     // voxel value bits, or the leaf's mask word holding the slot
  int4 o;        // leaf origin (or the gathered record's bits)
};
template <bool FUSE>
__device__ __forceinline__ void next_stage1(const TrainNet& TN, const TreeView& tv, int64_t j, NextSample& ns) {
  const SampleSpec& sp = TN.spec;
  if (j >= sp.n) return;
  if (!FUSE || !TN.fused) {
    ns.o = __builtin_bit_cast(int4, TN.xt[j]);
    return;
  }
  const uint64_t hsh = sm_mix(sp.step_seed + SM_GOLDEN * (uint64_t)(j + 1));
  const uint32_t g = (uint32_t)__umul64hi(hsh, (uint64_t)sp.npop);
  if (sp.src == SRC_VOXELS) {
    ns.key = tv.vox_key[g];
    ns.aux.x = __float_as_uint(tv.values[g]);
  } else {
    ns.key = g;
    const uint32_t leaf = g >> 9;
    ns.o = tv.leaf_o[leaf];
    ns.aux = *(const uint2*)&tv.leaf_mask[(size_t)leaf * 8 + ((g & 511u) >> 6)];
  }
}
template <bool FUSE>
__device__ __forceinline__ void next_stage2(const TrainNet& TN, const TreeView& tv, int64_t j, NextSample& ns) {
  if (FUSE && j < TN.spec.n && TN.fused && TN.spec.src == SRC_VOXELS) ns.o = tv.leaf_o[ns.key >> 9];
}
template <bool FUSE>
__device__ __forceinline__ void next_sample(const TrainNet& TN, const NextSample& ns, Smp& s) {
  const SampleSpec& sp = TN.spec;
  if (!FUSE || !TN.fused) {
    const floatx4 r = __builtin_bit_cast(floatx4, ns.o);
    s.x[0] = r[0];
    s.x[1] = r[1];
    s.x[2] = r[2];
    s.t = r[3];
    s.cls = (int)r[3];
    return;
  }
  const uint32_t n0 = ns.key & 511u;
  const int px = ns.o.x + (int)(n0 >> 6), py = ns.o.y + (int)((n0 >> 3) & 7u), pz = ns.o.z + (int)(n0 & 7u);
  s.x[0] = ((float)(px - sp.lo[0]) + 0.5f) * sp.inv_d;
  s.x[1] = ((float)(py - sp.lo[1]) + 0.5f) * sp.inv_d;
  s.x[2] = ((float)(pz - sp.lo[2]) + 0.5f) * sp.inv_d;
  if (sp.src == SRC_VOXELS) {
    s.t = __uint_as_float(ns.aux.x) * sp.tscale;
  } else {
    const uint64_t w = ((uint64_t)ns.aux.y << 32) | ns.aux.x;
    s.t = (float)((w >> (n0 & 63u)) & 1ull);
  }
  s.cls = 0;
}

// gamma(x) into S layout.  Feature f < m is cos(2 pi b_f.x) = sin(2 pi (b_f.x + 1/4)),
// m <= f < 2m is sin(2 pi b_{f-m}.x), f >= 2m is zero padding.  The hardware sine
// takes revolutions; the phase is reduced with fract first.  The FP32 form forms the
// phase in double precision so the feature is accurate to the sine's own error.
// benc holds b_f as float4 rows (x, y, z, 0).
template <int PREC>
__device__ __forceinline__ float phase(const floatx4& b, const Smp& s, float shift) {
  if constexpr (PREC == NVDB_FP32) {
    double u = (double)b[0] * s.x[0] + (double)b[1] * s.x[1] + (double)b[2] * s.x[2] + (double)shift;
    return (float)(u - floor(u));
  } else {
    return __builtin_amdgcn_fractf(fmaf(b[0], s.x[0], fmaf(b[1], s.x[1], fmaf(b[2], s.x[2], shift))));
  }
}
template <int PREC, int NIB>
__device__ __forceinline__ void encode_S(const Smp& s, const float* benc, int m, uint32_t (&X)[NIB][PR<PREC>::SR]) {
  const int h = lane_id() >> 5;
  if (2 * m == 32 * NIB) {
    // cos features fill the first half of the blocks and the sin features of the same
    // frequencies the second half, in the same registers: one phase per pair
#pragma unroll
    for (int t = 0; t < NIB / 2; ++t) {
      floatx16 vc, vs;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const floatx4 b = *(const floatx4*)(benc + 4 * sfeat(t, r, h));
        vc[r] = __builtin_amdgcn_sinf(phase<PREC>(b, s, 0.25f));
        vs[r] = __builtin_amdgcn_sinf(phase<PREC>(b, s, 0.f));
      }
      PR<PREC>::store(vc, X[t]);
      PR<PREC>::store(vs, X[t + NIB / 2]);
    }
  } else {
#pragma unroll
    for (int t = 0; t < NIB; ++t) {
      floatx16 v;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = sfeat(t, r, h);
        int fi = f < m ? f : f - m;
        fi = fi < m ? fi : 0;
        const floatx4 b = *(const floatx4*)(benc + 4 * fi);
        const float val = __builtin_amdgcn_sinf(phase<PREC>(b, s, f < m ? 0.25f : 0.f));
        v[r] = (f < 2 * m) ? val : 0.f;
      }
      PR<PREC>::store(v, X[t]);
    }
  }
}

// Phases u_f = b_f . x of the 2m = 32 NIB fast path on the FP32 matrix cores:
// 32x32x2 products with A = (b_f components) and B = (x components) put u for
// frequency 32 tb + 8 (r / 4) + 4 h + r mod 4 of the lane's sample in register r,
// which is the S layout of the cos block tb and the sin block tb + NIB/2.
// The k index is the coordinate component: lane half h carries components h and
// 2 + h (the fourth component of every row of B is zero).
template <int NIB>
struct PhaseA {
  float a[NIB / 2][2];
  __device__ __forceinline__ void load(const float* benc) {
    const int l = lane_id(), h = l >> 5, fl = l & 31;
#pragma unroll
    for (int tb = 0; tb < NIB / 2; ++tb) {
      a[tb][0] = benc[4 * (32 * tb + fl) + h];
      a[tb][1] = benc[4 * (32 * tb + fl) + 2 + h];
    }
  }
};
template <int NIB>
__device__ __forceinline__ void phases_mfma(const PhaseA<NIB>& A, const Smp& s, floatx16 (&u)[NIB / 2]) {
  const int h = lane_id() >> 5;
  const float b0 = h ? s.x[1] : s.x[0], b1 = h ? 0.f : s.x[2];
#pragma unroll
  for (int tb = 0; tb < NIB / 2; ++tb) {
    u[tb] = __builtin_amdgcn_mfma_f32_32x32x2f32(A.a[tb][0], b0, floatx16{}, 0, 0, 0);
    u[tb] = __builtin_amdgcn_mfma_f32_32x32x2f32(A.a[tb][1], b1, u[tb], 0, 0, 0);
  }
}
// gamma(x) of the fast path from MFMA phases, BF16 S-layout blocks.
template <int NIB>
__device__ __forceinline__ void encode_bf16_mfma(const PhaseA<NIB>& A, const Smp& s, uint32_t (&X)[NIB][8]) {
  floatx16 u[NIB / 2];
  phases_mfma<NIB>(A, s, u);
#pragma unroll
  for (int tb = 0; tb < NIB / 2; ++tb) {
    floatx16 vc, vs;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      vc[r] = __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(u[tb][r] + 0.25f));
      vs[r] = __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(u[tb][r]));
    }
    PR<NVDB_BF16>::store(vc, X[tb]);
    PR<NVDB_BF16>::store(vs, X[tb + NIB / 2]);
  }
}

// ------------------------------------------------------------ LDS addressing
// bf16 rows (weights and exchanged activations) are 256 bytes long; the 8-byte
// chunk c of row r is stored at chunk c ^ swz(r).  Every access pattern below
// splits into a compile-time part and a lane part whose bits are disjoint, so
// the swizzled byte offset is (CT << 3) ^ lane_constant plus an immediate:
//   row-wise reads and row writes:  lane constant s*256 + ((swz(s) ^ h) << 3), s = lane & 31;
//   transposing reads (4 rows x 32 columns per 16-lane group):
//     lane constant (4h + (k>>2))*256 + ((((4gg + (k&3)) ^ (8(k>>2) + h))) << 3).
struct LaneK {
  uint32_t fwd, tr;
  int h, fl;
};
__device__ __forceinline__ LaneK lane_consts() {
  const int l = lane_id(), h = l >> 5, fl = l & 31, k = l & 15, gg = (l >> 4) & 1;
  LaneK K;
  K.h = h;
  K.fl = fl;
  K.fwd = (uint32_t)fl * 256u + ((uint32_t)(swz(fl) ^ h) << 3);
  const uint32_t lanebits = (uint32_t)((4 * gg + (k & 3)) ^ (8 * (k >> 2) + h));
  K.tr = (uint32_t)(4 * h + (k >> 2)) * 256u + (lanebits << 3);
  return K;
}

// A fragment of the forward product from LDS rows: output block ob (32 rows),
// k-step kk of input block t.  Elements [c0, c0+4) and [c0+8, c0+12) of row
// 32 ob + i, c0 = 32t + 16kk + 4h.
// Rows of consecutive 32-row blocks lie `bstride` bytes apart (8192, or more where a
// block is padded so that the same lane's reads of two blocks do not share banks).
__device__ __forceinline__ bf16x8 frag_fwd(const char* rows, const LaneK& K, int ob, int t, int kk,
                                           int bstride = 32 * 256) {
  const char* base = rows + ob * bstride;
  const uint32_t o0 = ((uint32_t)(8 * t + 4 * kk) << 3) ^ K.fwd;
  const uint32_t o1 = ((uint32_t)(8 * t + 4 * kk + 2) << 3) ^ K.fwd;
  u32x2 a = *(const u32x2*)(base + o0);
  u32x2 b = *(const u32x2*)(base + o1);
  u32x4 v = {a[0], a[1], b[0], b[1]};
  return __builtin_bit_cast(bf16x8, v);
}
// Transposing read: lane (i, h) receives rows rbase + 8p + 4h + e (e < 4, p < 2) of
// column 32 cb + i, as 8 values ordered (p, e).  rbase is a multiple of 16.
__device__ __forceinline__ bf16x8 frag_tr(const char* rows, const LaneK& K, int rbase, int cb) {
  const int kb = (rbase >> 4) & 1;
  const char* base = rows + rbase * 256;
  const uint32_t o0 = ((uint32_t)(8 * cb + 4 * kb) << 3) ^ K.tr;
  const uint32_t o1 = ((uint32_t)(8 * cb + 4 * kb + 2) << 3) ^ K.tr;
  u32x2 a = lds_tr((const __bf16*)(base + o0));
  u32x2 b = lds_tr((const __bf16*)(base + 8 * 256 + o1));
  u32x4 v = {a[0], a[1], b[0], b[1]};
  return __builtin_bit_cast(bf16x8, v);
}
// The lane's S-layout blocks of one sample as a swizzled bf16 row.
template <int NIB>
__device__ __forceinline__ void write_rows_bf16(char* rows, const LaneK& K, const uint32_t (&S)[NIB][8]) {
#pragma unroll
  for (int t = 0; t < NIB; ++t)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      u32x2 v = {S[t][2 * a], S[t][2 * a + 1]};
      *(u32x2*)(rows + ((((uint32_t)(8 * t + 2 * a)) << 3) ^ K.fwd)) = v;
    }
}
template <int NIB>
__device__ __forceinline__ void write_rows_f32(float* rows, int pitch, const LaneK& K, const uint32_t (&S)[NIB][16]) {
  float* base = rows + K.fl * pitch + 4 * K.h;
#pragma unroll
  for (int t = 0; t < NIB; ++t)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      floatx4 v = {__uint_as_float(S[t][4 * a]), __uint_as_float(S[t][4 * a + 1]), __uint_as_float(S[t][4 * a + 2]),
                   __uint_as_float(S[t][4 * a + 3])};
      *(floatx4*)(base + 32 * t + 8 * a) = v;
    }
}
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
// Sum of the 8 bf16 values of a fragment, accumulated in fp32 with the bf16 dot
// product against (1, 1).  Written as inline assembly: the compiler builtin was seen
// reading one source register four times when fed elements of a bit-cast vector.
__device__ __forceinline__ float frag_sum(bf16x8 f, float acc) {
  const u32x4 u = __builtin_bit_cast(u32x4, f);
  const uint32_t ones = 0x3f803f80u;
#pragma unroll
  for (int q = 0; q < 4; ++q) asm("v_dot2c_f32_bf16 %0, %1, %2" : "+v"(acc) : "v"(ones), "v"(u[q]));
  return acc;
}

// ------------------------------------------------------------ per-layer weights
// A fragment of W_l for the forward product: rows = output features of block ob,
// k-step kk of input block t.
template <int PREC, int W, int NIBL>
struct WFwd {
  const char* lds;         // bf16 rows of this layer in LDS
  const u32x4* gfrag;      // bf16 fragments of this layer in HBM
  const float* gcol;       // fp32: this layer transposed [Win][W] in HBM
  bool global;             // bf16: read the fragments from HBM instead of LDS
  const LaneK* K;
  int bstride = 32 * 256;  // bytes between 32-row blocks of the LDS copy
  __device__ __forceinline__ typename PR<PREC>::Frag operator()(int ob, int t, int kk) const {
    if constexpr (PREC == NVDB_BF16) {
      if (global) return __builtin_bit_cast(bf16x8, gfrag[((ob * NIBL + t) * 2 + kk) * 64 + 32 * K->h + K->fl]);
      return frag_fwd(lds, *K, ob, t, kk, bstride);
    } else {
      return gcol[(size_t)sfeat(t, kk, K->h) * W + 32 * ob + K->fl];
    }
  }
};
// A fragment of W_l^T for the backward product: rows = input features of block ib,
// k-step kk of output block t.
template <int PREC, int W>
struct WBwd {
  const char* lds;
  const float* grow;    // fp32: [W][W] row-major
  const LaneK* K;
  __device__ __forceinline__ typename PR<PREC>::Frag operator()(int ib, int t, int kk) const {
    if constexpr (PREC == NVDB_BF16) {
      return frag_tr(lds, *K, 32 * t + 16 * kk, ib);
    } else {
      return grow[(size_t)sfeat(t, kk, K->h) * W + 32 * ib + K->fl];
    }
  }
};

// Raw buffer resource of a device array of `bytes` bytes (out-of-range lanes read 0).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
// BF16 transposed fragments of one layer (backward product) read from HBM/L2
// with buffer loads: uniform resource and layer offset, a fixed 16-byte slot per
// lane, so no per-load address arithmetic.
template <int W>
struct WBwdBuf {
  __amdgpu_buffer_rsrc_t rsrc;
  int soff;  // byte offset of the layer's fragments (uniform)
  int voff;  // lane * 16
  __device__ __forceinline__ bf16x8 operator()(int ib, int t, int kk) const {
    return __builtin_bit_cast(
        bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff, soff + ((ib * (W / 32) + t) * 2 + kk) * 1024, 0));
  }
};

// Accumulator initialised with the bias of the lane's 16 output features.
__device__ __forceinline__ floatx16 bias_acc(const float* bias, const LaneK& K, int ob) {
  const floatx4* b = (const floatx4*)(bias + 32 * ob + 4 * K.h);
  floatx16 a;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    floatx4 v = b[2 * q];
    a[4 * q] = v[0];
    a[4 * q + 1] = v[1];
    a[4 * q + 2] = v[2];
    a[4 * q + 3] = v[3];
  }
  return a;
}

// One output block of a layer: sum over input blocks and k-steps, starting from acc.
template <int PREC, int NIB, class AF>
__device__ __forceinline__ floatx16 layer_block(const AF& af, int ob, const uint32_t (&X)[NIB][PR<PREC>::SR],
                                                floatx16 acc) {
  using P = PR<PREC>;
#pragma unroll
  for (int t = 0; t < NIB; ++t)
#pragma unroll
    for (int kk = 0; kk < P::KS; ++kk) acc = P::mma(af(ob, t, kk), P::sfrag(X[t], kk), acc);
  return acc;
}

// Two output blocks sharing each B operand: two independent accumulator chains keep
// the MFMA pipe busy while each chain waits on its previous result.
// The A fragments are fetched PF k-steps ahead of their use (software pipeline), so
// the load latency overlaps the MFMAs of the preceding steps.
template <int PREC, int NIB, class AF>
__device__ __forceinline__ void layer_block2(const AF& af, int ob, const uint32_t (&X)[NIB][PR<PREC>::SR],
                                             floatx16& acc0, floatx16& acc1) {
  using P = PR<PREC>;
  constexpr int NS = NIB * P::KS;
  constexpr int PF = (PREC == NVDB_BF16) ? (NS < 8 ? NS : 8) : 1;
  typename P::Frag fa[PF], fb[PF];
#pragma unroll
  for (int s = 0; s < PF; ++s) {
    fa[s] = af(ob, s / P::KS, s % P::KS);
    fb[s] = af(ob + 1, s / P::KS, s % P::KS);
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int t = s / P::KS, kk = s % P::KS;
    const auto b = P::sfrag(X[t], kk);
    const auto a0 = fa[s % PF], a1 = fb[s % PF];
    if (s + PF < NS) {
      fa[s % PF] = af(ob, (s + PF) / P::KS, (s + PF) % P::KS);
      fb[s % PF] = af(ob + 1, (s + PF) / P::KS, (s + PF) % P::KS);
    }
    acc0 = P::mma(a0, b, acc0);
    acc1 = P::mma(a1, b, acc1);
    // keep the scheduler from sinking the prefetch back next to its use
    if constexpr (PREC == NVDB_BF16) __builtin_amdgcn_sched_barrier(0);
  }
}

// Step schedule of the BF16 forward chain: layer l has NB/2 block pairs of
// nsl(l) k-steps each; steps are numbered through all layers.
template <int NIB0, int NB, int H>
struct FwdSteps {
  static constexpr int KS = PR<NVDB_BF16>::KS;
  static constexpr int nsl(int l) { return (l == 0 ? NIB0 : NB) * KS; }
  static constexpr int per_layer(int l) { return (NB / 2) * nsl(l); }
  static constexpr int total() {
    int t = 0;
    for (int l = 0; l < H; ++l) t += per_layer(l);
    return t;
  }
  static constexpr int layer(int g) {
    int l = 0;
    while (g >= per_layer(l)) g -= per_layer(l++);
    return l;
  }
  static constexpr int local(int g) {
    int l = 0;
    while (g >= per_layer(l)) g -= per_layer(l++);
    return g;
  }
  static constexpr int pair(int g) { return local(g) / nsl(layer(g)); }  // within the layer
  static constexpr int step(int g) { return local(g) % nsl(layer(g)); }
  static constexpr int gpair(int g) { return layer(g) * (NB / 2) + pair(g); }
  static constexpr int DEFER = 2;  // steps of the next pair that run before a pair's epilogue
  // The epilogue of the pair ending at step g may wait until step DEFER-1 of the
  // next pair if that pair's first DEFER steps do not read this pair's outputs.
  static constexpr bool deferred(int g) {
    if (g + 1 >= total()) return false;
    if (layer(g + 1) == layer(g)) return true;
    return (DEFER - 1) / KS < 2 * pair(g);
  }
};

// Hidden activation (App. on activation functions): ACT_RELU, or ACT_SIN,
// h = sin(w z) with the derivative factor d = w cos(w z) kept for the backward
// pass.  The hardware sine takes revolutions: the phase z w / (2 pi) (+ 1/4 for
// the cosine) is reduced with fract first, formed in double precision in the
// FP32 form.
struct ActC {
  float w;       // sin frequency
  float rev;     // w / (2 pi)
  double rev64;  // w / (2 pi), FP32 form
};
template <int PREC>
__device__ __forceinline__ float act_phase(float z, const ActC& ac, float shift) {
  if constexpr (PREC == NVDB_FP32) {
    const double u = (double)z * ac.rev64 + (double)shift;
    return (float)(u - floor(u));
  } else {
    return __builtin_amdgcn_fractf(fmaf(z, ac.rev, shift));
  }
}
// h = act(a) into s (S layout); with ACT_SIN and d non-null also d = w cos(w a).
template <int PREC, int ACT>
__device__ __forceinline__ void store_act(floatx16 a, uint32_t* s, uint32_t* d, const ActC& ac) {
  if constexpr (ACT == ACT_RELU) {
    store_relu<PREC>(a, s);
  } else {
    floatx16 hv, dv;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      hv[i] = __builtin_amdgcn_sinf(act_phase<PREC>(a[i], ac, 0.f));
      if (d) dv[i] = ac.w * __builtin_amdgcn_sinf(act_phase<PREC>(a[i], ac, 0.25f));
    }
    PR<PREC>::store(hv, s);
    if (d) PR<PREC>::store(dv, d);
  }
}
// Input gradient block: a times the activation's derivative, from the stored
// activation (ReLU: a > 0) or the stored factor d (sin), stored in S layout.
template <int PREC, int ACT>
__device__ __forceinline__ void store_grad(floatx16 a, uint32_t* s, const uint32_t* act, const uint32_t* d) {
  if constexpr (ACT == ACT_RELU) {
    store_masked<PREC>(a, s, act);
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if constexpr (PREC == NVDB_BF16) {
        a[2 * i] *= bf16_lo(d[i]);
        a[2 * i + 1] *= bf16_hi(d[i]);
      } else {
        a[2 * i] *= __uint_as_float(d[2 * i]);
        a[2 * i + 1] *= __uint_as_float(d[2 * i + 1]);
      }
    }
    PR<PREC>::store(a, s);
  }
}

// All hidden layers of the BF16 forward pass in one software pipeline: weight
// fragments (independent of the data) are fetched PF steps ahead through block
// pairs and layers, and the bias/activation/convert epilogue of a block pair
// overlaps the next pair's first products (two accumulator sets alternate).
// Ds receives the sin derivative factors (ACT_SIN).
template <int W, int H, int NIB0, int ACT, class F0, class FL, int HD>
__device__ __forceinline__ void forward_chain_bf16(const F0& wf0, const FL& wfl, const uint32_t (&X0)[NIB0][8],
                                                   uint32_t (&Hs)[H][W / 32][8], uint32_t (&Ds)[HD][W / 32][8],
                                                   const float* sm_bias, const LaneK& K, const ActC& ac) {
  using P = PR<NVDB_BF16>;
  constexpr int NB = W / 32, KS = P::KS;
  using S = FwdSteps<NIB0, NB, H>;
  constexpr int T = S::total();
  constexpr int PF = 8;
  P::Frag fa[PF], fb[PF];
  floatx16 acc[2][2];
  auto fetch = [&](auto gc, P::Frag& x, P::Frag& y) {
    constexpr int g = decltype(gc)::value;
    constexpr int l = S::layer(g), ob = 2 * S::pair(g), t = S::step(g) / KS, kk = S::step(g) % KS;
    if constexpr (l == 0) {
      x = wf0(ob, t, kk);
      y = wf0(ob + 1, t, kk);
    } else {
      const auto wf = wfl(IC<l>{});
      x = wf(ob, t, kk);
      y = wf(ob + 1, t, kk);
    }
  };
  static_for<0, PF>([&](auto gc) {
    constexpr int g = decltype(gc)::value;
    if constexpr (g < T) fetch(gc, fa[g], fb[g]);
  });
  static_for<0, T>([&](auto gc) {
    constexpr int g = decltype(gc)::value;
    constexpr int l = S::layer(g), p = S::pair(g), s = S::step(g), buf = S::gpair(g) & 1;
    if constexpr (s == 0) {
      acc[buf][0] = bias_acc(sm_bias + l * W, K, 2 * p);
      acc[buf][1] = bias_acc(sm_bias + l * W, K, 2 * p + 1);
    }
    const P::Frag a0 = fa[g % PF], a1 = fb[g % PF];
    if constexpr (g + PF < T) fetch(IC<g + PF>{}, fa[g % PF], fb[g % PF]);
    P::Frag b;
    if constexpr (l == 0) b = P::sfrag(X0[s / KS], s % KS);
    else b = P::sfrag(Hs[l - 1][s / KS], s % KS);
    acc[buf][0] = P::mma(a0, b, acc[buf][0]);
    acc[buf][1] = P::mma(a1, b, acc[buf][1]);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (s == S::DEFER - 1 && S::gpair(g) > 0) {
      constexpr int ge = g - S::DEFER;  // last step of the previous pair
      if constexpr (S::deferred(ge)) {
        constexpr int le = S::layer(ge), pe = S::pair(ge);
        store_act<NVDB_BF16, ACT>(acc[buf ^ 1][0], Hs[le][2 * pe], ACT ? Ds[ACT ? le : 0][2 * pe] : nullptr, ac);
        store_act<NVDB_BF16, ACT>(acc[buf ^ 1][1], Hs[le][2 * pe + 1], ACT ? Ds[ACT ? le : 0][2 * pe + 1] : nullptr, ac);
      }
    }
    if constexpr (s == S::nsl(l) - 1 && !S::deferred(g)) {
      store_act<NVDB_BF16, ACT>(acc[buf][0], Hs[l][2 * p], ACT ? Ds[ACT ? l : 0][2 * p] : nullptr, ac);
      store_act<NVDB_BF16, ACT>(acc[buf][1], Hs[l][2 * p + 1], ACT ? Ds[ACT ? l : 0][2 * p + 1] : nullptr, ac);
    }
  });
}

__device__ __forceinline__ void relu16(floatx16& a) {
#pragma unroll
  for (int r = 0; r < 16; ++r) a[r] = fmaxf(a[r], 0.f);
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

// Value of S-layout register r of a block (bf16 or fp32 storage).
template <int PREC>
__device__ __forceinline__ float sval(const uint32_t* s, int r) {
  if constexpr (PREC == NVDB_BF16) return (r & 1) ? bf16_hi(s[r >> 1]) : bf16_lo(s[r >> 1]);
  else return __uint_as_float(s[r]);
}

}  // namespace nvdb
