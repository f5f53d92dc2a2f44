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
#include "mlp_device.h"

namespace nvdb {

// ============================================================== training kernel
template <int PREC, int W, int H, int KP, int C>
struct TrainCfg {
  static constexpr int NB = W / 32, NIB0 = KP / 32, NSLOT = 2;
  // Layers whose dW stays in registers for the whole step (BF16 form); the others
  // fold each iteration's contribution into the work-group's partial row in HBM.
  static constexpr bool DWREG = (PREC == NVDB_BF16);
  // BF16: where the weight fragments of layers 1..H-1 come from (HBM/L2 or the LDS copy)
  // (forward fragments from HBM/L2 were measured 5 % faster per step than from the
  // LDS copy)
  static constexpr bool FWD_GLOBAL = true;
  // BF16: the forward pass as one software pipeline over all layers (two block
  // pairs per layer or more)
  static constexpr bool FWD_CHAIN = (PREC == NVDB_BF16) && W >= 128;
  // (measured on the 4x128 network: all but layer 0 resident is fastest; its few
  // spills cost less than folding another layer per tile, while holding layer 0
  // as well spills far more)
  static constexpr int DWREG_FROM = (W >= 128) ? 1 : 0;
  static constexpr bool reg_layer(int l) { return DWREG && l >= DWREG_FROM; }
  // BF16 4x128 with layers 1.. resident: layer 0's dW accumulates in LDS (a
  // wave-private fp32 region) instead of the partial row; the dX products then
  // read their weight fragments from HBM/L2, which frees the LDS weight copy.
  static constexpr bool DW0_LDS = DWREG && W >= 128 && DWREG_FROM == 1 && KP <= 128;
  static constexpr bool DX_HBM = DW0_LDS;
  static constexpr bool lds_layer(int l) { return DW0_LDS && l == 0; }
  static constexpr bool fold_layer(int l) { return !reg_layer(l) && !lds_layer(l); }
  static constexpr bool any_rmw = !DWREG || DWREG_FROM > (DW0_LDS ? 1 : 0);
  static constexpr int RB = (PREC == NVDB_BF16) ? 0 : (KP > W ? KP : W) + 4;  // fp32 row pitch (floats)
  static constexpr int ROWS_BYTES = (PREC == NVDB_BF16) ? 32 * 256 : 32 * RB * 4;
  // slot: G rows, input-activation rows, last-hidden-layer rows (head), gy [C][32].
  // The FP32 form keeps the last hidden layer's rows in a private buffer per wave
  // instead (written right after the forward pass) to free its registers.
  static constexpr bool HH_PRIVATE = (PREC != NVDB_BF16);
  // BF16: layer 0's input rows in panels of 128 features, each one 256-byte row per
  // sample; panel 0 follows the G rows, further panels follow gy.
  static constexpr int XPANELS = (PREC == NVDB_BF16 && KP > 128) ? KP / 128 : 1;
  static_assert(XPANELS == 1 || KP % 128 == 0, "input panels of 128 features");
  static constexpr int XP_OFF = (HH_PRIVATE ? 2 : 3) * ROWS_BYTES + 32 * C * 4;
  static constexpr int SLOT_BYTES = XP_OFF + (XPANELS - 1) * ROWS_BYTES;
  static __device__ __forceinline__ int xpanel(int p) { return p == 0 ? ROWS_BYTES : XP_OFF + (p - 1) * ROWS_BYTES; }
  static constexpr int HH_BYTES = HH_PRIVATE ? 4 * ROWS_BYTES : 0;
  static constexpr int WL_BYTES = (PREC == NVDB_BF16 && !DX_HBM) ? (H - 1) * W * 256 : 0;
  static constexpr int DW0_BYTES = DW0_LDS ? W * KP * 4 : 0;  // [wave][a][b][quad][lane][4] floats
  static constexpr int SMALL_FLOATS = H * W + C * W + 4 + 4 * (KP / 2) + 8;
  static constexpr int LDS_BYTES = WL_BYTES + NSLOT * SLOT_BYTES + HH_BYTES + SMALL_FLOATS * 4 + DW0_BYTES;
  // dW blocks owned by a wave: waves form a 2 x 2 grid over (output, input) blocks.
  static constexpr int OBW = NB / 2;
  static constexpr int IBW0 = NIB0 / 2, IBW = NB / 2;
  static constexpr int IBWMAX = IBW0 > IBW ? IBW0 : IBW;
  // the wave that sums the bias gradient of its output block a (spread over the two
  // waves of a row of the 2 x 2 grid when each owns two output blocks)
  static __device__ __forceinline__ bool bias_owner(int a, int wi) { return OBW == 1 ? wi == 0 : a == wi; }
};

template <int PREC, int W, int H, int KP, int C, int ACT>
__global__ void __launch_bounds__(256, 1) __attribute__((amdgpu_waves_per_eu(1, 1))) k_train(TrainLaunch L) {
  using P = PR<PREC>;
  using CF = TrainCfg<PREC, W, H, KP, C>;
  constexpr int NB = CF::NB, NIB0 = CF::NIB0, SR = P::SR, OBW = CF::OBW;
  constexpr bool BF = (PREC == NVDB_BF16);
  __shared__ __attribute__((aligned(16))) char smem[CF::LDS_BYTES];

  const TrainNet& TN = L.nets[blockIdx.y];
  if (TN.prev_loss && *TN.prev_loss < *TN.stop_below) return;  // uniform: this network has converged
  const NetView& nv = TN.net;
  const SampleSpec& sp = TN.spec;
  const int wave = wave_id();

  // ---- LDS carve-up
  char* wl0 = smem;                                                // bf16 layers 1..H-1
  char* slots0 = smem + CF::WL_BYTES;
  char* hh0 = slots0 + CF::NSLOT * CF::SLOT_BYTES;                  // FP32: per-wave rows of a_H
  float* sm_bias0 = (float*)(hh0 + CF::HH_BYTES);                    // [H][W]
  float* sm_whead0 = sm_bias0 + H * W;                              // [C][W]
  float* sm_bhead0 = sm_whead0 + C * W;                             // [C] (padded to 4)
  float* sm_benc0 = sm_bhead0 + 4;                                  // [KP/2][4]
  float* sm_red = sm_benc0 + 4 * (KP / 2);                          // [8] reductions
  float* dw0 = sm_red + 8;                                          // layer 0's dW (DW0_LDS)

  // ---- stage parameters
  if constexpr (BF) {
    const u32x4* src = (const u32x4*)((const char*)nv.wrow + (size_t)W * 256);  // skip layer 0
    u32x4* dst = (u32x4*)wl0;
    for (int i = threadIdx.x; i < CF::WL_BYTES / 16; i += blockDim.x) dst[i] = src[i];
  }
  for (int i = threadIdx.x; i < H * W; i += blockDim.x) sm_bias0[i] = nv.bias[i];
  for (int i = threadIdx.x; i < C * W; i += blockDim.x) sm_whead0[i] = nv.whead[i];
  if (threadIdx.x < C) sm_bhead0[threadIdx.x] = nv.bhead[threadIdx.x];
  for (int i = threadIdx.x; i < 4 * (KP / 2); i += blockDim.x) sm_benc0[i] = nv.benc[i];
  if constexpr (CF::DW0_LDS)
    for (int i = threadIdx.x; i < CF::DW0_BYTES / 16; i += blockDim.x) ((floatx4*)dw0)[i] = floatx4{0.f, 0.f, 0.f, 0.f};
  __syncthreads();

  // ---- per-wave accumulators kept across iterations
  floatx16 dacc[H][OBW][CF::IBWMAX];
#pragma unroll
  for (int l = 0; l < H; ++l)
#pragma unroll
    for (int a = 0; a < OBW; ++a)
#pragma unroll
      for (int b = 0; b < CF::IBWMAX; ++b) dacc[l][a][b] = floatx16{};
  float dbias[H][OBW];
#pragma unroll
  for (int l = 0; l < H; ++l)
#pragma unroll
    for (int a = 0; a < OBW; ++a) dbias[l][a] = 0.f;
  float dwh[C], dbh[C];
#pragma unroll
  for (int c = 0; c < C; ++c) dwh[c] = dbh[c] = 0.f;
  float loss_acc = 0.f;

  const int wo = wave >> 1, wi = wave & 1;
  const int64_t n_iter = (sp.n + 127) / 128;
  float* partial = TN.partial + (size_t)blockIdx.x * nv.s.pstride();

  PhaseA<NIB0> pa;
  const bool fastenc = BF && 2 * nv.nfreq == 32 * NIB0;
  if (fastenc) pa.load(sm_benc0);
  NextSample nx{};
  {
    const int64_t j0 = (int64_t)blockIdx.x * 128 + wave * 32 + (lane_id() & 31);
    next_stage1<BF>(TN, TN.tree, j0, nx);
    next_stage2<BF>(TN, TN.tree, j0, nx);
  }
  for (int64_t it = blockIdx.x; it < n_iter; it += L.G) {
    const NextSample cur = nx;
    const int64_t jn = (it + L.G) * 128 + wave * 32 + (lane_id() & 31);
    next_stage1<BF>(TN, TN.tree, jn, nx);
    const LaneK K = lane_consts();
    const int h = K.h, fl = K.fl;
    const int z = opaque_zero();
    const float* sm_bias = sm_bias0 + z;
    const float* sm_whead = sm_whead0 + z;
    const float* sm_bhead = sm_bhead0 + z;
    const float* sm_benc = sm_benc0 + z;
    const char* wl = wl0 + z;
    char* slots = slots0 + z;
    const bool first = (it == (int64_t)blockIdx.x);  // first iteration stores into the partial row
    const int64_t j = it * 128 + wave * 32 + fl;
    Smp smp;
    smp.valid = j < sp.n;
    next_sample<BF>(TN, cur, smp);

    // ================= forward
    uint32_t Hs[H][NB][SR];  // Hs[l] = a_{l+1} (S layout), l = 0..H-1
    uint32_t Ds[ACT ? H : 1][NB][SR];  // sin activation: derivative factors of the layers
    const ActC ac{nv.act_w, nv.act_rev, nv.act_rev64};
    {
      uint32_t X0[NIB0][SR];
      if constexpr (BF) {
        if (fastenc) encode_bf16_mfma<NIB0>(pa, smp, X0);
        else encode_S<PREC, NIB0>(smp, sm_benc, nv.nfreq, X0);
      } else {
        encode_S<PREC, NIB0>(smp, sm_benc, nv.nfreq, X0);
      }
      WFwd<PREC, W, NIB0> wf0{nullptr, (const u32x4*)nv.wfrag + z, (const float*)nv.wcol + z, true, &K};
      auto wfl = [&](auto lc) {
        constexpr int l = decltype(lc)::value;
        return WFwd<PREC, W, NB>{wl + (size_t)(l - 1) * W * 256,
                                 (const u32x4*)((const __bf16*)nv.wfrag + (size_t)W * KP + (size_t)(l - 1) * W * W) + z,
                                 (const float*)nv.wcol + z + (size_t)KP * W + (size_t)(l - 1) * W * W, CF::FWD_GLOBAL,
                                 &K};
      };
      if constexpr (CF::FWD_CHAIN) {
        forward_chain_bf16<W, H, NIB0, ACT>(wf0, wfl, X0, Hs, Ds, sm_bias, K, ac);
      } else {
#pragma unroll
        for (int ob = 0; ob < NB; ob += 2) {
          floatx16 a0 = bias_acc(sm_bias, K, ob), a1 = bias_acc(sm_bias, K, ob + 1);
          layer_block2<PREC, NIB0>(wf0, ob, X0, a0, a1);
          store_act<PREC, ACT>(a0, Hs[0][ob], ACT ? Ds[0][ob] : nullptr, ac);
          store_act<PREC, ACT>(a1, Hs[0][ob + 1], ACT ? Ds[0][ob + 1] : nullptr, ac);
        }
        static_for<1, H>([&](auto lc) {
          constexpr int l = decltype(lc)::value;
          const auto wf = wfl(lc);
#pragma unroll
          for (int ob = 0; ob < NB; ob += 2) {
            floatx16 a0 = bias_acc(sm_bias + l * W, K, ob), a1 = bias_acc(sm_bias + l * W, K, ob + 1);
            layer_block2<PREC, NB>(wf, ob, Hs[l - 1], a0, a1);
            store_act<PREC, ACT>(a0, Hs[l][ob], ACT ? Ds[ACT ? l : 0][ob] : nullptr, ac);
            store_act<PREC, ACT>(a1, Hs[l][ob + 1], ACT ? Ds[ACT ? l : 0][ob + 1] : nullptr, ac);
          }
        });
      }
    }
    next_stage2<BF>(TN, TN.tree, jn, nx);  // the next tile's leaf origin (voxels)
    // head (VALU): y_c = sum_f Wh[c][f] a_H[f] + bh[c]
    float y[C], gy[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      float acc = 0.f;
#pragma unroll
      for (int ob = 0; ob < NB; ++ob)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const floatx4 w4 = *(const floatx4*)(sm_whead + c * W + 32 * ob + 8 * q + 4 * h);
#pragma unroll
          for (int e = 0; e < 4; ++e) acc = fmaf(w4[e], sval<PREC>(Hs[H - 1][ob], 4 * q + e), acc);
        }
      y[c] = acc + shfl_xor32(acc) + sm_bhead[c];
    }
    const float Ls = loss_grad<C>(sp, smp, j, y, gy);
    if (h == 0) loss_acc += Ls;

    // g_H = (Wh^T gy) * act'(z_H)
    uint32_t Gc[NB][SR];
#pragma unroll
    for (int ob = 0; ob < NB; ++ob) {
      floatx16 g;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        floatx4 v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const floatx4 w4 = *(const floatx4*)(sm_whead + c * W + 32 * ob + 8 * q + 4 * h);
          v += w4 * gy[c];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) g[4 * q + e] = v[e];
      }
      store_grad<PREC, ACT>(g, Gc[ob], Hs[H - 1][ob], Ds[ACT ? H - 1 : 0][ob]);
    }
    if constexpr (CF::HH_PRIVATE) {
      // the previous iteration's readers of this buffer finished before its last barrier
      write_rows_f32<NB>((float*)(hh0 + z + wave * CF::ROWS_BYTES), CF::RB, K, Hs[H - 1]);
    }

    // ================= backward through the hidden layers
    static_for<0, H>([&](auto kc) {
      constexpr int l = H - 1 - decltype(kc)::value;
      constexpr int NIBl = (l == 0) ? NIB0 : NB;
      constexpr int IBWl = NIBl / 2;
      constexpr bool HEAD = (l == H - 1);
      // input activations a_l of layer l as rows (gamma recomputed for l = 0)
      uint32_t X0[NIB0][SR];
      if constexpr (l == 0) {
        if constexpr (BF) {
          if (fastenc) encode_bf16_mfma<NIB0>(pa, smp, X0);
          else encode_S<PREC, NIB0>(smp, sm_benc, nv.nfreq, X0);
        } else {
          encode_S<PREC, NIB0>(smp, sm_benc, nv.nfreq, X0);
        }
      }
      // layers folded into the partial row: fetch the running sums now so that the
      // loads complete under the exchange below
      constexpr bool PREFETCH = CF::fold_layer(l) && (BF ? l <= 1 : l == 0);  // where registers allow
      float prev[PREFETCH ? OBW : 1][PREFETCH ? CF::IBWMAX : 1][16];
      if constexpr (PREFETCH) {
        if (!first) {
          const int win = (l == 0) ? nv.s.win(0) : W;  // compile-time above layer 0
#pragma unroll
          for (int a = 0; a < OBW; ++a)
#pragma unroll
            for (int b = 0; b < CF::IBWMAX; ++b)
              if (b < IBWl) {
                const int ob = wo * OBW + a, ib = wi * IBWl + b, i = 32 * ib + fl;
                const float* p0 = partial + nv.s.woff(l) + (size_t)(32 * ob + 4 * h) * win + i;
#pragma unroll
                for (int r = 0; r < 16; ++r) prev[a][b][r] = (i < win) ? p0[(size_t)(8 * (r >> 2) + (r & 3)) * win] : 0.f;
              }
        }
      }

#pragma unroll
      for (int round = 0; round < 4 / CF::NSLOT; ++round) {
        const int my_slot = wave - round * CF::NSLOT;
        if (my_slot >= 0 && my_slot < CF::NSLOT) {
          char* sl = slots + my_slot * CF::SLOT_BYTES;
          if constexpr (BF) {
            write_rows_bf16<NB>(sl, K, Gc);
            if constexpr (l == 0) {
              constexpr int NP = NIB0 / CF::XPANELS;
              static_for<0, CF::XPANELS>([&](auto pc) {
                constexpr int pn = decltype(pc)::value;
                write_rows_bf16<NP>(sl + CF::xpanel(pn), K, *reinterpret_cast<const uint32_t(*)[NP][8]>(&X0[NP * pn]));
              });
            } else {
              write_rows_bf16<NB>(sl + CF::ROWS_BYTES, K, Hs[l - 1 < 0 ? 0 : l - 1]);
            }
            if constexpr (HEAD) write_rows_bf16<NB>(sl + 2 * CF::ROWS_BYTES, K, Hs[H - 1]);
          } else {
            write_rows_f32<NB>((float*)sl, CF::RB, K, Gc);
            if constexpr (l == 0) write_rows_f32<NIB0>((float*)(sl + CF::ROWS_BYTES), CF::RB, K, X0);
            else write_rows_f32<NB>((float*)(sl + CF::ROWS_BYTES), CF::RB, K, Hs[l - 1 < 0 ? 0 : l - 1]);
          }
          if constexpr (HEAD) {
            if (h == 0) {
              float* gyr = (float*)(sl + (CF::HH_PRIVATE ? 2 : 3) * CF::ROWS_BYTES);
#pragma unroll
              for (int c = 0; c < C; ++c) gyr[c * 32 + fl] = gy[c];
            }
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
              if constexpr (BF) ga[a] = frag_tr(sl, K, 16 * kk, ob);
              else ga[a] = ((const float*)sl)[(2 * kk + h) * CF::RB + 32 * ob + fl];
              if (CF::bias_owner(a, wi)) {  // bias gradient: column sums of g over the samples
                if constexpr (BF) dbias[l][a] = frag_sum(ga[a], dbias[l][a]);
                else dbias[l][a] += ga[a];
              }
            }
#pragma unroll
            for (int b = 0; b < CF::IBWMAX; ++b) {
              if (b < IBWl) {
                const int ib = wi * IBWl + b;
                if constexpr (BF) {
                  if constexpr (l == 0 && CF::XPANELS > 1) {
                    constexpr int NP = NIB0 / CF::XPANELS;
                    hb[b] = frag_tr(sl + CF::xpanel(ib / NP), K, 16 * kk, ib % NP);
                  } else {
                    hb[b] = frag_tr(sl + CF::ROWS_BYTES, K, 16 * kk, ib);
                  }
                }
                if constexpr (!BF) hb[b] = ((const float*)(sl + CF::ROWS_BYTES))[(2 * kk + h) * CF::RB + 32 * ib + fl];
              }
            }
#pragma unroll
            for (int a = 0; a < OBW; ++a)
#pragma unroll
              for (int b = 0; b < CF::IBWMAX; ++b)
                if (b < IBWl) dacc[l][a][b] = P::mma(ga[a], hb[b], dacc[l][a][b]);
            if constexpr (HEAD) {
              // head weights and bias: wave w owns the head's input block w (if it exists)
              const float* gyr = (const float*)(sl + (CF::HH_PRIVATE ? 2 : 3) * CF::ROWS_BYTES);
              if (wave < NB) {
                if constexpr (BF) {
                  const bf16x8 hh = frag_tr(sl + 2 * CF::ROWS_BYTES, K, 16 * kk, wave);
                  const u32x4 u = __builtin_bit_cast(u32x4, hh);
#pragma unroll
                  for (int c = 0; c < C; ++c) {
                    const floatx4 g0 = *(const floatx4*)(gyr + c * 32 + 16 * kk + 4 * h);
                    const floatx4 g1 = *(const floatx4*)(gyr + c * 32 + 16 * kk + 8 + 4 * h);
                    float acc = dwh[c];
                    acc = fmaf(g0[0], bf16_lo(u[0]), acc);
                    acc = fmaf(g0[1], bf16_hi(u[0]), acc);
                    acc = fmaf(g0[2], bf16_lo(u[1]), acc);
                    acc = fmaf(g0[3], bf16_hi(u[1]), acc);
                    acc = fmaf(g1[0], bf16_lo(u[2]), acc);
                    acc = fmaf(g1[1], bf16_hi(u[2]), acc);
                    acc = fmaf(g1[2], bf16_lo(u[3]), acc);
                    acc = fmaf(g1[3], bf16_hi(u[3]), acc);
                    dwh[c] = acc;
                    if (wave == 0) dbh[c] += ((g0[0] + g0[1]) + (g0[2] + g0[3])) + ((g1[0] + g1[1]) + (g1[2] + g1[3]));
                  }
                } else {
                  const float* hhr = (const float*)(hh0 + z + (round * CF::NSLOT + sl_i) * CF::ROWS_BYTES);
                  const float hv = hhr[(2 * kk + h) * CF::RB + 32 * wave + fl];
#pragma unroll
                  for (int c = 0; c < C; ++c) {
                    const float g = gyr[c * 32 + 2 * kk + h];
                    dwh[c] = fmaf(g, hv, dwh[c]);
                    if (wave == 0) dbh[c] += g;
                  }
                }
              }
            }
          }
        }
        __syncthreads();
      }

      if constexpr (CF::lds_layer(l)) {
        // add this iteration's blocks to the wave's region of layer 0's dW in LDS
#pragma unroll
        for (int a = 0; a < OBW; ++a)
#pragma unroll
          for (int b = 0; b < CF::IBWMAX; ++b) {
            if (b < IBWl) {
              floatx4* q = (floatx4*)(dw0 + z) + ((wave * OBW + a) * IBWl + b) * 256 + lane_id();
#pragma unroll
              for (int qd = 0; qd < 4; ++qd) {
                floatx4 v = q[64 * qd];
                v[0] += dacc[l][a][b][4 * qd];
                v[1] += dacc[l][a][b][4 * qd + 1];
                v[2] += dacc[l][a][b][4 * qd + 2];
                v[3] += dacc[l][a][b][4 * qd + 3];
                q[64 * qd] = v;
              }
              dacc[l][a][b] = floatx16{};
            }
          }
      }
      if constexpr (CF::fold_layer(l)) {
        // fold this iteration's blocks into the work-group's partial row.  Every
        // running sum is loaded before the first store: a store may alias a later
        // load as far as the compiler knows, so interleaving them would cost one
        // memory round trip per element.
        const int win = (l == 0) ? nv.s.win(0) : W;
        float old[PREFETCH ? 1 : OBW][PREFETCH ? 1 : CF::IBWMAX][16];
        if constexpr (!PREFETCH) {
#pragma unroll
          for (int a = 0; a < OBW; ++a)
#pragma unroll
            for (int b = 0; b < CF::IBWMAX; ++b)
              if (b < IBWl) {
                const int ob = wo * OBW + a, ib = wi * IBWl + b, i = 32 * ib + fl;
                const float* p0 = partial + nv.s.woff(l) + (size_t)(32 * ob + 4 * h) * win + i;
#pragma unroll
                for (int r = 0; r < 16; ++r)
                  old[a][b][r] = (!first && i < win) ? p0[(size_t)(8 * (r >> 2) + (r & 3)) * win] : 0.f;
              }
        }
#pragma unroll
        for (int a = 0; a < OBW; ++a)
#pragma unroll
          for (int b = 0; b < CF::IBWMAX; ++b) {
            if (b < IBWl) {
              const int ob = wo * OBW + a, ib = wi * IBWl + b, i = 32 * ib + fl;
              float* p0 = partial + nv.s.woff(l) + (size_t)(32 * ob + 4 * h) * win + i;
              if (i < win) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                  float* q = p0 + (size_t)(8 * (r >> 2) + (r & 3)) * win;
                  float old_v;
                  if constexpr (PREFETCH) old_v = first ? 0.f : prev[a][b][r];
                  else old_v = old[a][b][r];
                  *q = old_v + dacc[l][a][b][r];
                }
              }
              dacc[l][a][b] = floatx16{};
            }
          }
      }

      if constexpr (l > 0) {
        // g_l = (W_l^T g_{l+1}) * act'(z_l)
        WBwd<PREC, W> wb_p{wl + (size_t)(l - 1) * W * 256,
                           (const float*)nv.wrow + z + (size_t)W * KP + (size_t)(l - 1) * W * W, &K};
        const WBwdBuf<W> wb_b{raw_rsrc(nv.wtfrag, BF ? wtfrag_elems(nv.s) * 2 : 0), z + (l - 1) * W * W * 2,
                              lane_id() * 16};
        uint32_t Gn[NB][SR];
#pragma unroll
        for (int ib = 0; ib < NB; ib += 2) {
          floatx16 a0 = floatx16{}, a1 = floatx16{};
          if constexpr (BF && CF::DX_HBM) layer_block2<PREC, NB>(wb_b, ib, Gc, a0, a1);
          else layer_block2<PREC, NB>(wb_p, ib, Gc, a0, a1);
          store_grad<PREC, ACT>(a0, Gn[ib], Hs[l - 1][ib], Ds[ACT ? l - 1 : 0][ib]);
          store_grad<PREC, ACT>(a1, Gn[ib + 1], Hs[l - 1][ib + 1], Ds[ACT ? l - 1 : 0][ib + 1]);
        }
#pragma unroll
        for (int ib = 0; ib < NB; ++ib)
#pragma unroll
          for (int q = 0; q < SR; ++q) Gc[ib][q] = Gn[ib][q];
      }
    });
  }

  // ---- write this work-group's partial gradient row
  const int h = lane_id() >> 5, fl = lane_id() & 31;
  if constexpr (CF::any_rmw) {
    // a work-group without iterations still owes zeros in the rows it would have accumulated
    if ((int64_t)blockIdx.x >= n_iter) {
      static_for<0, H>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        if constexpr (CF::fold_layer(l)) {
          const int64_t n_el = (int64_t)W * nv.s.win(l);
          for (int64_t q = threadIdx.x; q < n_el; q += blockDim.x) partial[nv.s.woff(l) + q] = 0.f;
        }
      });
    }
  }
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
  if constexpr (CF::DW0_LDS) {
    // layer 0's dW from the wave's LDS region (every work-group writes its row)
    const int win = nv.s.win(0);
#pragma unroll
    for (int a = 0; a < OBW; ++a)
#pragma unroll
      for (int b = 0; b < NIB0 / 2; ++b) {
        const int ob = wo * OBW + a, ib = wi * (NIB0 / 2) + b, i = 32 * ib + fl;
        const floatx4* q = (const floatx4*)dw0 + ((wave * OBW + a) * (NIB0 / 2) + b) * 256 + lane_id();
        if (i < win) {
#pragma unroll
          for (int qd = 0; qd < 4; ++qd) {
            const floatx4 v = q[64 * qd];
#pragma unroll
            for (int e = 0; e < 4; ++e) partial[(size_t)sfeat(ob, 4 * qd + e, h) * win + i] = v[e];
          }
        }
      }
  }
  // biases (waves of the first input column own them) and head: combine the lane halves
#pragma unroll
  for (int l = 0; l < H; ++l)
#pragma unroll
    for (int a = 0; a < OBW; ++a) {
      const float v = dbias[l][a] + shfl_xor32(dbias[l][a]);
      if (CF::bias_owner(a, wi) && h == 0) partial[nv.s.boff(l) + 32 * (wo * OBW + a) + fl] = v;
    }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const float v = dwh[c] + shfl_xor32(dwh[c]);
    if (wave < NB && h == 0) partial[nv.s.woff(H) + (size_t)c * W + 32 * wave + fl] = v;
    const float b = dbh[c] + shfl_xor32(dbh[c]);
    if (wave == 0 && lane_id() == 0) partial[nv.s.boff(H) + c] = b;
  }
  // loss: fixed-order reduction over the wave, then over the four waves
  float v = loss_acc;
#pragma unroll
  for (int off = 16; off >= 1; off >>= 1) {
    int src = (lane_id() ^ off) << 2;
    v += __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v)));
  }
  if (lane_id() == 0) sm_red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) TN.loss_partial[blockIdx.x] = ((sm_red[0] + sm_red[1]) + sm_red[2]) + sm_red[3];
}

// ============================================================== inference kernel
// A decode tile shape: WV waves per work-group (one LDS copy of the weights), each
// NTV 32-sample tiles sharing every weight fragment.
template <int PREC, int W, int H, int KP, int C, int NTV = 1, int WV = INFER_WAVES>
struct InferCfg {
  static constexpr int NT = NTV;
  static constexpr int WAVES = WV;
  // Each 32-row block of the weight copy is followed by 64 pad bytes: a lane's reads of
  // two blocks 8192 bytes apart would hit the same banks when fetched together.
  static constexpr int BSTRIDE = 32 * 256 + 64;
  static constexpr int WL_BYTES = (PREC == NVDB_BF16) ? H * (W / 32) * BSTRIDE : 0;
  static constexpr int SMALL_FLOATS = H * W + C * W + 4 + 4 * (KP / 2);
  static constexpr int LDS_BYTES = WL_BYTES + SMALL_FLOATS * 4;
};

// The decode work of one work-group: one network's weights staged in LDS, then
// passes of NT 32-sample tiles per wave.
template <int PREC, int W, int H, int KP, int C, int ACT, int NTV, int WV>
struct InferWG {
  using P = PR<PREC>;
  using CF = InferCfg<PREC, W, H, KP, C, NTV, WV>;
  static constexpr int NB = W / 32, NIB0 = KP / 32, SR = P::SR, NT = CF::NT;
  static constexpr int NA = NB > NIB0 ? NB : NIB0;
  static constexpr bool BF = (PREC == NVDB_BF16);
  char* wl0;
  float* sm_bias0;
  float* sm_whead0;
  float* sm_bhead0;
  float* sm_benc0;
  __device__ __forceinline__ explicit InferWG(char* smem)
      : wl0(smem),
        sm_bias0((float*)(smem + CF::WL_BYTES)),
        sm_whead0(sm_bias0 + H * W),
        sm_bhead0(sm_whead0 + C * W),
        sm_benc0(sm_bhead0 + 4) {}
  // Copies network nv's weights into LDS; every thread of the work-group takes part,
  // and the caller synchronises before (if LDS was in use) and after.
  __device__ __forceinline__ void stage(const NetView& nv) const {
    if constexpr (BF) {
      const u32x4* src = (const u32x4*)nv.wrow;
      for (int i = threadIdx.x; i < H * W * 16; i += blockDim.x) {  // 16-byte pieces of the 256-byte rows
        const int row = i >> 4, blk = row >> 5;
        *(u32x4*)(wl0 + blk * CF::BSTRIDE + (row & 31) * 256 + (i & 15) * 16) = src[i];
      }
    }
    for (int i = threadIdx.x; i < H * W; i += blockDim.x) sm_bias0[i] = nv.bias[i];
    for (int i = threadIdx.x; i < C * W; i += blockDim.x) sm_whead0[i] = nv.whead[i];
    if (threadIdx.x < C) sm_bhead0[threadIdx.x] = nv.bhead[threadIdx.x];
    for (int i = threadIdx.x; i < 4 * (KP / 2); i += blockDim.x) sm_benc0[i] = nv.benc[i];
  }
  // One wave's tiles of samples base + 32 u (u < NT) of sp, written as I directs.
  __device__ __forceinline__ void pass(const NetView& nv, const ActC& ac, const PhaseA<NIB0>& pa, bool fastenc,
                                       const SampleSpec& sp, const TreeView& tv, const InferLaunch& I,
                                       int64_t base) const {
    const LaneK K = lane_consts();
    const int h = K.h, fl = K.fl;
    const int z = opaque_zero();
    const float* sm_bias = sm_bias0 + z;
    const float* sm_whead = sm_whead0 + z;
    const float* sm_bhead = sm_bhead0 + z;
    const float* sm_benc = sm_benc0 + z;
    const char* wl = wl0 + z;
    uint32_t A[NT][NA][SR];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const Smp smp = fetch_sample(sp, tv, base + 32 * u + fl, h == 0);
      uint32_t X0[NIB0][SR];
      if constexpr (BF) {
        if (fastenc) encode_bf16_mfma<NIB0>(pa, smp, X0);
        else encode_S<PREC, NIB0>(smp, sm_benc, nv.nfreq, X0);
      } else {
        encode_S<PREC, NIB0>(smp, sm_benc, nv.nfreq, X0);
      }
#pragma unroll
      for (int t = 0; t < NIB0; ++t)
#pragma unroll
        for (int q = 0; q < SR; ++q) A[u][t][q] = X0[t][q];
    }
    static_for<0, H>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      constexpr int NIBl = (l == 0) ? NIB0 : NB;
      WFwd<PREC, W, NIBl> wf{wl + (size_t)l * (W / 32) * CF::BSTRIDE,
                             (const u32x4*)((const __bf16*)nv.wfrag + (l == 0 ? 0 : (size_t)W * KP + (size_t)(l - 1) * W * W)) + z,
                             (const float*)nv.wcol + z + (l == 0 ? 0 : (size_t)KP * W + (size_t)(l - 1) * W * W),
                             BF && l == 0 && KP > ROW_ELEMS, &K, CF::BSTRIDE};
      uint32_t Bn[NT][NB][SR];
#pragma unroll
      for (int ob = 0; ob < NB; ++ob) {
        floatx16 acc[NT];
        const floatx16 b0 = bias_acc(sm_bias + l * W, K, ob);
#pragma unroll
        for (int u = 0; u < NT; ++u) acc[u] = b0;
#pragma unroll
        for (int t = 0; t < NIBl; ++t) {
#pragma unroll
          for (int kk = 0; kk < P::KS; ++kk) {
            typename P::Frag af = wf(ob, t, kk);
#pragma unroll
            for (int u = 0; u < NT; ++u) acc[u] = P::mma(af, P::sfrag(A[u][t], kk), acc[u]);
          }
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) store_act<PREC, ACT>(acc[u], Bn[u][ob], nullptr, ac);
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
          for (int q = 0; q < 4; ++q) {
            const floatx4 w4 = *(const floatx4*)(sm_whead + c * W + 32 * ob + 8 * q + 4 * h);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc = fmaf(w4[e], sval<PREC>(A[u][ob], 4 * q + e), acc);
          }
        y[u][c] = acc + shfl_xor32(acc) + sm_bhead[c];
      }
    // outputs
    if (I.out_kind == OUT_MASK) {
      // one 32-bit word per 32-slot tile (the mask words are little-endian uint64)
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const uint32_t bits = (uint32_t)(__ballot(y[u][0] > 0.f) & 0xffffffffull);
        if (lane_id() == 0 && base + 32 * u < sp.n) ((uint32_t*)I.mask)[(base + 32 * u) >> 5] = bits;
      }
    } else {
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const int64_t j = base + 32 * u + fl;
        if (h == 0 && j < sp.n) {
          if (I.out_kind == OUT_VALUES) {
            I.y[j] = y[u][0] * I.out_scale;
          } else if (I.out_kind == OUT_SCATTER) {
#pragma unroll
            for (int c = 0; c < C; ++c) I.y[(size_t)I.yidx[j] * C + c] = y[u][c] * I.out_scale;
          } else if (I.out_kind == OUT_CLASS) {
            int best = 0;
            float bv = y[u][0];
#pragma unroll
            for (int c = 1; c < C; ++c)
              if (y[u][c] > bv) {
                bv = y[u][c];
                best = c;
              }
            I.cls[j] = (uint8_t)best;
          } else {
#pragma unroll
            for (int c = 0; c < C; ++c) I.y[(size_t)j * C + c] = y[u][c];
          }
        }
      }
    }
  }
};

template <int PREC, int W, int H, int KP, int C, int ACT, int NTV, int WV>
__global__ void __launch_bounds__(64 * WV, 1) __attribute__((amdgpu_waves_per_eu(WV / 4, WV / 4)))
k_infer(InferLaunch I) {
  using WG = InferWG<PREC, W, H, KP, C, ACT, NTV, WV>;
  __shared__ __attribute__((aligned(16))) char smem[WG::CF::LDS_BYTES];
  const NetView& nv = I.net;
  SampleSpec sp = I.spec;
  if (sp.n_dev) sp.n = min(sp.n, (int64_t)*sp.n_dev);  // count known only on the device
  const ActC ac{nv.act_w, nv.act_rev, nv.act_rev64};
  const WG wg(smem);
  wg.stage(nv);
  __syncthreads();
  PhaseA<WG::NIB0> pa;
  const bool fastenc = WG::BF && 2 * nv.nfreq == 32 * WG::NIB0;
  if (fastenc) pa.load(wg.sm_benc0);
  const int64_t per_wave = 32 * WG::NT;
  const int64_t stride = (int64_t)gridDim.x * WV * per_wave;
  for (int64_t base = ((int64_t)blockIdx.x * WV + wave_id()) * per_wave; base < sp.n; base += stride)
    wg.pass(nv, ac, pa, fastenc, sp, I.tree, I, base);
}

// Decode of many networks of one shape in one launch (the experts of a domain
// decomposition).  Their samples sit in one array, each network's run starting on
// a chunk boundary (a chunk is one pass of a work-group, WV x NT x 32 samples);
// work-group b takes the chunks [b n / G, (b + 1) n / G) of the n chunks and
// restages the weights whenever its chunk belongs to another network.  Outputs
// are scattered: yslot[yidx[s]] = y(s) * out_scale of the network.
template <int PREC, int W, int H, int KP, int C, int ACT, int NTV, int WV>
__global__ void __launch_bounds__(64 * WV, 1) __attribute__((amdgpu_waves_per_eu(WV / 4, WV / 4)))
k_infer_group(InferGroupLaunch M) {
  using WG = InferWG<PREC, W, H, KP, C, ACT, NTV, WV>;
  __shared__ __attribute__((aligned(16))) char smem[WG::CF::LDS_BYTES];
  constexpr int64_t CH = 32 * (int64_t)WG::NT * WV;
  const WG wg(smem);
  const uint32_t nc = M.chunk_start[M.n_nets];
  const uint32_t c0 = (uint32_t)((uint64_t)blockIdx.x * nc / gridDim.x);
  const uint32_t c1 = (uint32_t)((uint64_t)(blockIdx.x + 1) * nc / gridDim.x);
  int cur = -1, k = 0;
  PhaseA<WG::NIB0> pa;
  bool fastenc = false;
  for (uint32_t c = c0; c < c1; ++c) {
    while (k + 1 < M.n_nets && M.chunk_start[k + 1] <= c) ++k;  // chunks are ordered by network
    const NetView& nv = M.nets[k].net;
    if (k != cur) {
      if (cur >= 0) __syncthreads();
      wg.stage(nv);
      __syncthreads();
      fastenc = WG::BF && 2 * nv.nfreq == 32 * WG::NIB0;
      if (fastenc) pa.load(wg.sm_benc0);
      cur = k;
    }
    const int64_t first = (int64_t)c * CH;  // sample offset of the chunk
    SampleSpec sp{};
    sp.src = SRC_COORDS;
    sp.direct = 1;
    sp.coords = M.x + 3 * first;
    sp.n = min(CH, (int64_t)M.chunk_start[k] * CH + M.count[k] - first);
    InferLaunch I{};
    I.out_kind = OUT_SCATTER;
    I.out_scale = M.nets[k].out_scale;
    I.y = M.yslot;
    I.yidx = M.slot + first;
    const ActC ac{nv.act_w, nv.act_rev, nv.act_rev64};
    wg.pass(nv, ac, pa, fastenc, sp, TreeView{}, I, (int64_t)wave_id() * 32 * WG::NT);
  }
}

// ============================================================== FP8 (e4m3) forward
// The FP8 form of the forward pass (decoding): every hidden layer multiplies
// e4m3 weights, quantised per layer with s_w = 448 / max|W|, by e4m3 inputs,
// quantised per sample with s_a = 448 / max_f |h_f|, on the gfx950
// 32x32x64 FP8 MFMA with FP32 accumulation; z = acc / (s_w s_a) + b, ReLU; the
// head runs on the FP32 activations.  Values are clamped to +-448 before the
// conversion, which rounds to nearest even.
//
// Operand layout of the 32x32x64 FP8 MFMA: lane (i, g) of A holds row i, bytes
// s = 0..31 of k-group g; lane (j, g) of B holds column j with the same k
// assignment, so a k index is any (g, s) pair used consistently by A and B.
// The B operand of k-step kk is the pair of S-layout blocks 2kk, 2kk+1 of the
// lane's sample, 16 bytes each, so byte s of lane half g carries feature
//   f(kk, g, s) = 32 (2kk + s/16) + 8 ((s mod 16) / 4) + 4 g + s mod 4,
// and the weight fragments are stored with the same assignment:
//   [layer][ob][kk][plane p][lane][16 bytes], bytes 16p .. 16p+15 of the lane.
__device__ __forceinline__ int fp8_feature(int kk, int g, int s) {
  return 32 * (2 * kk + (s >> 4)) + 8 * ((s & 15) >> 2) + 4 * g + (s & 3);
}
// Four values to e4m3 (round to nearest even).  Callers scale by 448 / max|x|,
// so no value exceeds 448 by more than a rounding of the product, far below the
// first value the conversion does not saturate (464): the clamp of the
// definition never acts and is not executed.
__device__ __forceinline__ uint32_t pack4_fp8(float a, float b, float c, float d) {
  uint32_t w = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(c, d, (int)w, true);
}

// Per-layer scales: one work-group per hidden layer.
__global__ void __launch_bounds__(256) k_fp8_scales(NetShape s, const float* theta, float* w8inv, float* w8scale) {
  const int l = blockIdx.x;
  const int64_t n = (int64_t)s.W * s.win(l);
  const float* w = theta + s.woff(l);
  float mx = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) mx = fmaxf(mx, fabsf(w[i]));
  __shared__ float red[256];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float sc = red[0] > 0.f ? 448.f / red[0] : 1.f;
    w8scale[l] = sc;
    w8inv[l] = 1.f / sc;
  }
}
// One thread per 4 fragment bytes.
__global__ void __launch_bounds__(256) k_fp8_pack(NetShape s, const float* theta, const float* w8scale, char* w8) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // dword index
  const int64_t total = fp8_weight_bytes(s) / 4;
  if (q >= total) return;
  // locate the layer
  int64_t off = q * 4;
  int l = 0;
  int64_t lbytes = (int64_t)s.W * s.KP;
  while (off >= lbytes) {
    off -= lbytes;
    ++l;
    lbytes = (int64_t)s.W * s.W;
  }
  const int winp = (l == 0) ? s.KP : s.W, win = s.win(l), ks = winp / 64;
  const int frag = (int)(off / 2048), rem = (int)(off % 2048);
  const int ob = frag / ks, kk = frag % ks;
  const int p = rem / 1024, lane = (rem % 1024) / 16, s0 = 16 * p + (rem % 16);
  const int i = 32 * ob + (lane & 31), g = lane >> 5;
  const float sc = w8scale[l];
  float v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int f = fp8_feature(kk, g, s0 + e);
    v[e] = f < win ? theta[s.woff(l) + (int64_t)i * win + f] * sc : 0.f;
  }
  ((uint32_t*)w8)[q] = pack4_fp8(v[0], v[1], v[2], v[3]);
}

template <int W, int H, int KP, int C>
struct Infer8Cfg {
  static constexpr int NT = INFER8_NT;
  static constexpr int WAVES = INFER8_WAVES;
  static constexpr int WL_BYTES = W * KP + (H - 1) * W * W;
  static constexpr int SMALL_FLOATS = H * W + C * W + 4 + 4 * (KP / 2) + 4;
  static constexpr int LDS_BYTES = WL_BYTES + SMALL_FLOATS * 4;
};

// gamma(x) in S layout, FP32 values (any m <= 16 NIB).
template <int NIB>
__device__ __forceinline__ void encode_f32(const Smp& s, const float* benc, int m, float (&X)[NIB][16]) {
  const int h = lane_id() >> 5;
  if (2 * m == 32 * NIB) {
    // cos and sin of the same frequency sit in blocks t and t + NIB/2, same register
#pragma unroll
    for (int t = 0; t < NIB / 2; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const floatx4 b = *(const floatx4*)(benc + 4 * sfeat(t, r, h));
        const float u = fmaf(b[0], s.x[0], fmaf(b[1], s.x[1], b[2] * s.x[2]));
        X[t][r] = __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(u + 0.25f));
        X[t + NIB / 2][r] = __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(u));
      }
    return;
  }
#pragma unroll
  for (int t = 0; t < NIB; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int f = sfeat(t, r, h);
      int fi = f < m ? f : f - m;
      fi = fi < m ? fi : 0;
      const floatx4 b = *(const floatx4*)(benc + 4 * fi);
      const float val = __builtin_amdgcn_sinf(phase<NVDB_BF16>(b, s, f < m ? 0.25f : 0.f));
      X[t][r] = (f < 2 * m) ? val : 0.f;
    }
}

template <int C, int NT>
__device__ __forceinline__ void write_outputs(const InferLaunch& I, const float (&y)[NT][C], int64_t base, int fl,
                                              int h) {
  const SampleSpec& sp = I.spec;
  if (I.out_kind == OUT_MASK) {
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const uint32_t bits = (uint32_t)(__ballot(y[u][0] > 0.f) & 0xffffffffull);
      if (lane_id() == 0 && base + 32 * u < sp.n) ((uint32_t*)I.mask)[(base + 32 * u) >> 5] = bits;
    }
    return;
  }
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
          if (y[u][c] > bv) {
            bv = y[u][c];
            best = c;
          }
        I.cls[j] = (uint8_t)best;
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) I.y[(size_t)j * C + c] = y[u][c];
      }
    }
  }
}

template <int W, int H, int KP, int C>
__global__ void __launch_bounds__(64 * INFER8_WAVES, INFER8_WGS)
    __attribute__((amdgpu_waves_per_eu(INFER8_WAVES / 4 * INFER8_WGS, INFER8_WAVES / 4 * INFER8_WGS)))
    k_infer_fp8(InferLaunch I) {
  using CF = Infer8Cfg<W, H, KP, C>;
  constexpr int NB = W / 32, NIB0 = KP / 32, NT = CF::NT;
  constexpr int NA = NB > NIB0 ? NB : NIB0;
  __shared__ __attribute__((aligned(16))) char smem[CF::LDS_BYTES];
  const NetView& nv = I.net;
  SampleSpec sp = I.spec;
  if (sp.n_dev) sp.n = min(sp.n, (int64_t)*sp.n_dev);  // count known only on the device
  const int wave = wave_id();

  char* wl0 = smem;
  float* sm_bias0 = (float*)(smem + CF::WL_BYTES);
  float* sm_whead0 = sm_bias0 + H * W;
  float* sm_bhead0 = sm_whead0 + C * W;
  float* sm_benc0 = sm_bhead0 + 4;
  float* sm_winv0 = sm_benc0 + 4 * (KP / 2);
  {
    const u32x4* src = (const u32x4*)I.w8;
    u32x4* dst = (u32x4*)wl0;
    for (int i = threadIdx.x; i < CF::WL_BYTES / 16; i += blockDim.x) dst[i] = src[i];
  }
  for (int i = threadIdx.x; i < H * W; i += blockDim.x) sm_bias0[i] = nv.bias[i];
  for (int i = threadIdx.x; i < C * W; i += blockDim.x) sm_whead0[i] = nv.whead[i];
  if (threadIdx.x < C) sm_bhead0[threadIdx.x] = nv.bhead[threadIdx.x];
  for (int i = threadIdx.x; i < 4 * (KP / 2); i += blockDim.x) sm_benc0[i] = nv.benc[i];
  if (threadIdx.x < H) sm_winv0[threadIdx.x] = I.w8inv[threadIdx.x];
  __syncthreads();

  PhaseA<NIB0> pa;
  const bool fastenc = 2 * nv.nfreq == 32 * NIB0;
  if (fastenc) pa.load(sm_benc0);
  const int64_t per_wave = 32 * NT;
  const int64_t stride = (int64_t)gridDim.x * CF::WAVES * per_wave;
  for (int64_t base = ((int64_t)blockIdx.x * CF::WAVES + wave) * per_wave; base < sp.n; base += stride) {
    const int lane = lane_id();
    const int h = lane >> 5, fl = lane & 31;
    const int z = opaque_zero();
    const float* sm_bias = sm_bias0 + z;
    const float* sm_whead = sm_whead0 + z;
    const float* sm_bhead = sm_bhead0 + z;
    const float* sm_benc = sm_benc0 + z;
    const float* sm_winv = sm_winv0 + z;
    const char* wl = wl0 + z;
    const LaneK K = lane_consts();
    float Z[NT][NA][16];
    float zmax[NT];  // per-sample max of the current activations (lane's half)
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      zmax[u] = 0.f;
      const Smp smp = fetch_sample(sp, I.tree, base + 32 * u + fl, h == 0);
      float X0[NIB0][16];
      if (fastenc) {
        floatx16 ph[NIB0 / 2];
        phases_mfma<NIB0>(pa, smp, ph);
#pragma unroll
        for (int tb = 0; tb < NIB0 / 2; ++tb)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            X0[tb][r] = __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(ph[tb][r] + 0.25f));
            X0[tb + NIB0 / 2][r] = __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(ph[tb][r]));
          }
      } else {
        encode_f32<NIB0>(smp, sm_benc, nv.nfreq, X0);
      }
#pragma unroll
      for (int t = 0; t < NIB0; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) Z[u][t][r] = X0[t][r];
    }
    static_for<0, H>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      constexpr int NIBl = (l == 0) ? NIB0 : NB;
      constexpr int KSl = NIBl / 2;
      constexpr int LOFF = (l == 0) ? 0 : W * KP + (l - 1) * W * W;
      // per-sample quantisation of the layer input
      uint32_t Bq[NT][NIBl][4];
      float inv_sa[NT];
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        float mx = zmax[u];
        if constexpr (l == 0) {
#pragma unroll
          for (int t = 0; t < NIBl; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) mx = fmaxf(mx, fabsf(Z[u][t][r]));
        }
        mx = fmaxf(mx, shfl_xor32(mx));
        const float sa = mx > 0.f ? 448.f / mx : 1.f;
        inv_sa[u] = 1.f / sa;
#pragma unroll
        for (int t = 0; t < NIBl; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            Bq[u][t][q] = pack4_fp8(Z[u][t][4 * q] * sa, Z[u][t][4 * q + 1] * sa, Z[u][t][4 * q + 2] * sa,
                                    Z[u][t][4 * q + 3] * sa);
      }
      const float winv = sm_winv[l];
#pragma unroll
      for (int u = 0; u < NT; ++u) zmax[u] = 0.f;
#pragma unroll
      for (int ob = 0; ob < NB; ++ob) {
        floatx16 acc[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u) acc[u] = floatx16{};
#pragma unroll
        for (int kk = 0; kk < KSl; ++kk) {
          const char* fr = wl + LOFF + (ob * KSl + kk) * 2048 + lane * 16;
          const u32x4 a0 = *(const u32x4*)fr;
          const u32x4 a1 = *(const u32x4*)(fr + 1024);
          const intx8 A = {(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3],
                           (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
#pragma unroll
          for (int u = 0; u < NT; ++u) {
            const intx8 Bv = {(int)Bq[u][2 * kk][0], (int)Bq[u][2 * kk][1], (int)Bq[u][2 * kk][2], (int)Bq[u][2 * kk][3],
                              (int)Bq[u][2 * kk + 1][0], (int)Bq[u][2 * kk + 1][1], (int)Bq[u][2 * kk + 1][2],
                              (int)Bq[u][2 * kk + 1][3]};
            acc[u] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, Bv, acc[u], 0, 0, 0, 0, 0, 0);
          }
        }
        const floatx16 b0 = bias_acc(sm_bias + l * W, K, ob);
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          const float d = winv * inv_sa[u];
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            Z[u][ob][r] = fmaxf(fmaf(acc[u][r], d, b0[r]), 0.f);
            zmax[u] = fmaxf(zmax[u], Z[u][ob][r]);  // ReLU outputs: |z| = z
          }
        }
      }
    });
    // head on the FP32 activations
    float y[NT][C];
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        float acc = 0.f;
#pragma unroll
        for (int ob = 0; ob < NB; ++ob)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const floatx4 w4 = *(const floatx4*)(sm_whead + c * W + 32 * ob + 8 * q + 4 * h);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc = fmaf(w4[e], Z[u][ob][4 * q + e], acc);
          }
        y[u][c] = acc + shfl_xor32(acc) + sm_bhead[c];
      }
    write_outputs<C, NT>(I, y, base, fl, h);
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
    // 256-byte rows (the LDS image): layer 0 only when its inputs fit one row
    __bf16* rows = (__bf16*)A.wrow + (size_t)l * s.W * ROW_ELEMS;
    if (l > 0 || s.KP <= ROW_ELEMS) rows[(size_t)o * ROW_ELEMS + swz_elem(o, i)] = (__bf16)th;
    {
      // forward A fragment (ob, t, kk): lane (r, g) element e holds
      // W[32 ob + r][32 t + 16 kk + 8 (e >> 2) + 4 g + (e & 3)]
      const int nib = (l == 0 ? s.KP : s.W) / 32;
      const size_t lbase = (l == 0) ? 0 : (size_t)s.W * s.KP + (size_t)(l - 1) * s.W * s.W;
      const int ob = o >> 5, ii = o & 31, t = i >> 5, rem = i & 31, kk = rem >> 4, rr = rem & 15;
      const int e = ((rr >> 3) << 2) | (rr & 3), hh = (rr >> 2) & 1;
      const int lane = ii + 32 * hh;
      ((__bf16*)A.wfrag)[lbase + ((((size_t)ob * nib + t) * 2 + kk) * 64 + lane) * 8 + e] = (__bf16)th;
    }
    if (l > 0) {
      // transposed fragment (ib, t, kk) of the input-gradient product: lane (r, g)
      // element q holds W[32 t + 16 kk + 8 (q >> 2) + 4 g + (q & 3)][32 ib + r]
      const int nb = s.W / 32;
      const size_t lbase = (size_t)(l - 1) * s.W * s.W;
      const int ib = i >> 5, ii = i & 31, t = o >> 5, rem = o & 31, kk = rem >> 4, rr = rem & 15;
      const int q = ((rr >> 3) << 2) | (rr & 3), hh = (rr >> 2) & 1;
      const int lane = ii + 32 * hh;
      ((__bf16*)A.wtfrag)[lbase + ((((size_t)ib * nb + t) * 2 + kk) * 64 + lane) * 8 + q] = (__bf16)th;
    }
  } else {
    const size_t loff = (l == 0) ? 0 : (size_t)s.KP * s.W + (size_t)(l - 1) * s.W * s.W;
    ((float*)A.wrow)[loff + (size_t)o * (l == 0 ? s.KP : s.W) + i] = th;
    ((float*)A.wcol)[loff + (size_t)i * s.W + o] = th;
  }
}

// One work-group per 64 parameters: its four waves each sum a quarter of the
// work-group partial rows (four interleaved running sums per lane keep eight
// loads in flight), then wave 0 combines the quarters in a fixed order, so the
// result is the same on every run.
constexpr int RED_P = 64;
__global__ void __launch_bounds__(256) k_reduce_adam(AdamLaunch AL) {
  const AdamNet& A = AL.nets[blockIdx.y];
  const int64_t P = A.s.nparams(), R = A.s.pstride();
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t p = (int64_t)blockIdx.x * RED_P + lane;
  if (A.prev_loss && *A.prev_loss < *A.stop_below) {  // skipped step: carry the loss forward
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (A.loss_out) *A.loss_out = *A.prev_loss;
      if (A.ran) *A.ran = 0;
    }
    return;
  }
  if ((int64_t)blockIdx.x * RED_P >= P) return;  // uniform per work-group
  if (blockIdx.x == 0 && threadIdx.x == 0 && A.ran) *A.ran = 1;
  if (blockIdx.x == 0 && threadIdx.x < 64 && A.loss_out) {
    // step loss: lane-strided sums of the work-group losses, then a butterfly over
    // the wave; lane 0's result follows the same order on every run
    float L = 0.f;
    for (int g = threadIdx.x; g < A.G; g += 64) L += A.loss_partial[g];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) L += __shfl_xor(L, off);
    if (threadIdx.x == 0) *A.loss_out = L * A.loss_scale;
  }
  __shared__ float red[4][RED_P];
  const int per = (A.G + 3) / 4;
  const int g0 = q * per, g1 = min(A.G, g0 + per);
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  if (p < P) {
    const float* col = A.partial + p;
    int g = g0;
    for (; g + 8 <= g1; g += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = col[(size_t)(g + u) * R];
      s0 += v[0] + v[4];
      s1 += v[1] + v[5];
      s2 += v[2] + v[6];
      s3 += v[3] + v[7];
    }
    for (; g < g1; ++g) s0 += col[(size_t)g * R];
  }
  red[q][lane] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (q != 0 || p >= P) return;
  const float g = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
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

// Samples of one step, gathered once into (x, y, z, target or class) so that the
// fused kernel reads one coalesced 16-byte record per sample.
__global__ void __launch_bounds__(256) k_gather(SampleSpec sp, TreeView tv, floatx4* out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= sp.n) return;
  const Smp s = fetch_sample(sp, tv, j);
  out[j] = floatx4{s.x[0], s.x[1], s.x[2], sp.src == SRC_L1_SLOTS ? (float)s.cls : s.t};
}

// The samples of every network of one training launch in a single launch
// (blockIdx.y = network).
struct GatherLaunch {
  SampleSpec sp[NVDB_MAX_NETS];
  floatx4* out[NVDB_MAX_NETS];
};
__global__ void __launch_bounds__(256) k_gather_multi(GatherLaunch GL, TreeView tv) {
  const SampleSpec& sp = GL.sp[blockIdx.y];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= sp.n) return;
  const Smp s = fetch_sample(sp, tv, j);
  GL.out[blockIdx.y][j] = floatx4{s.x[0], s.x[1], s.x[2], sp.src == SRC_L1_SLOTS ? (float)s.cls : s.t};
}

__global__ void k_fill(float* p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_sample(uint64_t sseed, uint32_t npop, int64_t n, uint32_t* out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = (uint32_t)__umul64hi(sm_mix(sseed + SM_GOLDEN * (uint64_t)(j + 1)), (uint64_t)npop);
}

// ============================================================== host dispatch

template <int PREC, int W, int H, int KP, int C, int ACT>
KernelSet make_set() {
  static_assert(KP % 64 == 0, "the FP8 form takes k-steps of 64 features");
  KernelSet k{};
  k.train = k.train_classic = k_train<PREC, W, H, KP, C, ACT>;
  k.train_lds = TrainCfg<PREC, W, H, KP, C>::LDS_BYTES;
  k.infer_lds = InferCfg<PREC, W, H, KP, C>::LDS_BYTES;
  k.infer8 = ACT == ACT_RELU ? k_infer_fp8<W, H, KP, C> : nullptr;
  // decode tile shapes (waves per work-group, tiles per wave), the default first:
  // BF16 (8, 2), (8, 1), (4, 2), (4, 4); FP32 (8, 1), (4, 1), (4, 2)
  if constexpr (PREC == NVDB_BF16) {
    k.infer_group = k_infer_group<PREC, W, H, KP, C, ACT, 2, 8>;
    k.group_waves = 8;
    k.group_chunk = 32 * 2 * 8;
    k.infer_v[0] = {k_infer<PREC, W, H, KP, C, ACT, 2, 8>, 8, 2};
    k.infer_v[1] = {k_infer<PREC, W, H, KP, C, ACT, 1, 8>, 8, 1};
    k.infer_v[2] = {k_infer<PREC, W, H, KP, C, ACT, 2, 4>, 4, 2};
    k.infer_v[3] = {k_infer<PREC, W, H, KP, C, ACT, 4, 4>, 4, 4};
    k.n_infer_v = 4;
  } else {
    k.infer_group = k_infer_group<PREC, W, H, KP, C, ACT, 1, 8>;
    k.group_waves = 8;
    k.group_chunk = 32 * 1 * 8;
    k.infer_v[0] = {k_infer<PREC, W, H, KP, C, ACT, 1, 8>, 8, 1};
    k.infer_v[1] = {k_infer<PREC, W, H, KP, C, ACT, 1, 4>, 4, 1};
    k.infer_v[2] = {k_infer<PREC, W, H, KP, C, ACT, 2, 4>, 4, 2};
    k.n_infer_v = 3;
  }
  k.infer_sel = 0;
  if constexpr (PREC == NVDB_BF16 && W == 128 && KP == 128 && C == 1 && (H == 3 || H == 4) && ACT == ACT_RELU)
    k.train_rows = train_rows_kernel(H);
  return k;
}

// Shapes with compiled kernels: (W, H, KP, C), ReLU.
#define NVDB_FOR_SHAPES(X) \
  X(64, 3, 64, 1)          \
  X(64, 4, 128, 3)         \
  X(128, 4, 128, 1)        \
  X(128, 3, 128, 1)

bool find_kernels(int prec, int W, int H, int KP, int C, int act, KernelSet* out) {
  if (act == ACT_RELU) {
#define NVDB_MATCH(w, hh, kp, c)                                              \
  if (W == w && H == hh && KP == kp && C == c) {                              \
    *out = prec == NVDB_BF16 ? make_set<NVDB_BF16, w, hh, kp, c, ACT_RELU>()  \
                             : make_set<NVDB_FP32, w, hh, kp, c, ACT_RELU>(); \
    return true;                                                              \
  }
    NVDB_FOR_SHAPES(NVDB_MATCH)
#undef NVDB_MATCH
    // Fourier features as many as the width (m = W = 128, K = 256), BF16 form only:
    // the FP32 form's 256-float input rows do not fit the LDS next to its other buffers
    if (prec == NVDB_BF16 && W == 128 && H == 3 && KP == 256 && C == 1) {
      *out = make_set<NVDB_BF16, 128, 3, 256, 1, ACT_RELU>();
      return true;
    }
    return false;
  }
  // sin activation: the small 3x64 network in both forms and the 3x128 network with
  // m = 128 Fourier features in the BF16 form
  if (act == ACT_SIN) {
    if (W == 64 && H == 3 && KP == 64 && C == 1) {
      *out = prec == NVDB_BF16 ? make_set<NVDB_BF16, 64, 3, 64, 1, ACT_SIN>()
                               : make_set<NVDB_FP32, 64, 3, 64, 1, ACT_SIN>();
      return true;
    }
    if (prec == NVDB_BF16 && W == 128 && H == 3 && KP == 256 && C == 1) {
      *out = make_set<NVDB_BF16, 128, 3, 256, 1, ACT_SIN>();
      return true;
    }
  }
  return false;
}

void launch_train(const KernelSet& ks, const TrainLaunch& L, int n_nets, hipStream_t st) {
  hipLaunchKernelGGL(ks.train, dim3(L.G, n_nets), dim3(256), 0, st, L);
  NVDB_HIP(hipGetLastError());
}
int infer_grid(const KernelSet& ks, int64_t n) {
  // half a pass of the grid per work-group (idle waves help small decodes), at most
  // 4096 waves in flight
  const InferVariant& v = ks.infer_v[ks.infer_sel];
  const int64_t per_wg = 16 * (int64_t)v.nt * v.waves;
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + per_wg - 1) / per_wg, 4096 / v.waves));
}
void launch_infer_group(const KernelSet& ks, const InferGroupLaunch& M, hipStream_t st) {
  // one 8-wave work-group per compute unit, each taking a contiguous chunk range
  // (staging the weights once per network it meets); those past the chunk count exit
  hipLaunchKernelGGL(ks.infer_group, dim3(2048 / ks.group_waves), dim3(64 * ks.group_waves), 0, st, M);
  NVDB_HIP(hipGetLastError());
}
void launch_infer(const KernelSet& ks, const InferLaunch& I, int grid, hipStream_t st) {
  const InferVariant& v = ks.infer_v[ks.infer_sel];
  hipLaunchKernelGGL(v.fn, dim3(grid), dim3(64 * v.waves), 0, st, I);
  NVDB_HIP(hipGetLastError());
}
void launch_reduce_adam(const AdamLaunch& A, int64_t max_p, int n_nets, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_adam, dim3((unsigned)((max_p + RED_P - 1) / RED_P), n_nets), dim3(256), 0, st, A);
  NVDB_HIP(hipGetLastError());
}
void launch_write_shadow(const AdamNet& A, hipStream_t st) {
  hipLaunchKernelGGL(k_write_shadow, dim3((unsigned)((A.s.nparams() + 255) / 256)), dim3(256), 0, st, A);
  NVDB_HIP(hipGetLastError());
}
void launch_gather(const SampleSpec& sp, const TreeView& tv, floatx4* out, hipStream_t st) {
  if (sp.n <= 0) return;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((sp.n + 255) / 256)), dim3(256), 0, st, sp, tv, out);
  NVDB_HIP(hipGetLastError());
}
void launch_gather_multi(const SampleSpec* sp, floatx4* const* out, int n, const TreeView& tv, hipStream_t st) {
  GatherLaunch GL{};
  int64_t nmax = 0;
  for (int k = 0; k < n; ++k) {
    GL.sp[k] = sp[k];
    GL.out[k] = out[k];
    nmax = std::max<int64_t>(nmax, sp[k].n);
  }
  if (nmax <= 0) return;
  hipLaunchKernelGGL(k_gather_multi, dim3((unsigned)((nmax + 255) / 256), n), dim3(256), 0, st, GL, tv);
  NVDB_HIP(hipGetLastError());
}
void launch_quant_fp8(const NetShape& s, const float* theta, char* w8, float* w8inv, hipStream_t st) {
  float* scale = w8inv + s.H;  // the caller's buffer holds 2 H floats: 1/s_w, then s_w
  hipLaunchKernelGGL(k_fp8_scales, dim3(s.H), dim3(256), 0, st, s, theta, w8inv, scale);
  NVDB_HIP(hipGetLastError());
  const int64_t dw = fp8_weight_bytes(s) / 4;
  hipLaunchKernelGGL(k_fp8_pack, dim3((unsigned)((dw + 255) / 256)), dim3(256), 0, st, s, theta, (const float*)scale, w8);
  NVDB_HIP(hipGetLastError());
}
void launch_infer8(const KernelSet& ks, const InferLaunch& I, int grid, hipStream_t st) {
  hipLaunchKernelGGL(ks.infer8, dim3(grid), dim3(64 * INFER8_WAVES), 0, st, I);
  NVDB_HIP(hipGetLastError());
}
void launch_fill(float* p, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  NVDB_HIP(hipGetLastError());
}
void launch_sample(uint64_t sseed, uint32_t npop, int64_t n, uint32_t* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_sample, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sseed, npop, n, out);
  NVDB_HIP(hipGetLastError());
}

}  // namespace nvdb
