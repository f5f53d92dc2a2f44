// BF16 training kernel of the 128-wide coordinate MLPs that keeps activations as
// LDS rows (NeuralVDB Sec. 3.2, 3.3.1: the forward, loss and hand-derived backward
// of the networks replacing the lower tree levels).  Compiled with matrix-product
// results in general-purpose vector registers: the weight gradients, which live
// in the accumulation registers for the whole launch, are the only products
// written there, through an explicit operand constraint.
#include "mlp_device.h"

namespace nvdb {

// ======================================================= training kernel, activation rows
// BF16 form of the 128-wide networks on 128 Fourier features (m = 64) with one
// output.  Unlike k_train, which keeps every layer's activations in registers
// for the backward pass, the forward pass writes each hidden layer's bf16
// activations as swizzled sample rows to LDS as soon as they are formed: those
// rows are both the second operand of the layer above's weight gradient (the
// batch is the contraction dimension, read with transposing loads) and the
// source of the ReLU derivative.  That frees the registers that held them, so
// the weight gradients of all H layers accumulate in the accumulation registers
// for the whole launch (256 of them for H = 4).  One backward stage per layer:
// every wave writes its gradient rows, a barrier, each wave forms its 2 x 2
// blocks of dW over the work-group's 128 samples, interleaved with its own
// input-gradient products, then a barrier before the rows are rewritten.  The
// head's weight gradient comes from the last hidden layer's rows and the output
// gradients, staged the same way.  Weight fragments come from L2 through
// buffer loads (uniform resource and offsets, no per-load address arithmetic).
template <int H>
struct TrainRCfg {
  static constexpr int W = 128, KP = 128, NB = 4, NIB0 = 4;
  static constexpr int ROWS = 32 * 256;   // one wave's 32 sample rows (bf16, 256 bytes each)
  static constexpr int LROWS = 4 * ROWS;  // the work-group's 128 rows of one layer
  // rows of a_1 .. a_{H-1} (a_l = output of hidden layer l), then the gradient
  // rows (the last hidden layer's rows during the head stage), output gradients
  static constexpr int G_OFF = (H - 1) * LROWS;
  static constexpr int GY_OFF = G_OFF + LROWS;
  static constexpr int SMALL_OFF = GY_OFF + 4 * 32 * 4;
  static constexpr int SMALL_FLOATS = H * W + W + 4 + 4 * (KP / 2) + 8;
  static constexpr int LDS_BYTES = SMALL_OFF + SMALL_FLOATS * 4;
};

// A lane's S-layout block t of one sample read back from its swizzled row.
__device__ __forceinline__ void read_row_block(const char* rows, const LaneK& K, int t, uint32_t (&S)[8]) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const u32x2 v = *(const u32x2*)(rows + ((((uint32_t)(8 * t + 2 * a)) << 3) ^ K.fwd));
    S[2 * a] = v[0];
    S[2 * a + 1] = v[1];
  }
}
__device__ __forceinline__ void write_row_block(char* rows, const LaneK& K, int t, const uint32_t (&S)[8]) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const u32x2 v = {S[2 * a], S[2 * a + 1]};
    *(u32x2*)(rows + ((((uint32_t)(8 * t + 2 * a)) << 3) ^ K.fwd)) = v;
  }
}

// BF16 fragments of one layer from L2 with buffer loads.  Forward (A = W_l rows):
// fragment (ob, t, kk) of the MFMA-order copy; backward (A = W_l^T): fragment
// (ib, t, kk) of the transposed copy.  Both are [block][k-step][lane][16 bytes].
struct WBuf {
  __amdgpu_buffer_rsrc_t rsrc;
  int soff;  // byte offset of the layer (uniform)
  int voff;  // lane * 16
  int nib;   // input blocks of the layer (forward) or output blocks (backward)
  // The fragment's offset splits into a 4 KiB page (scalar offset, shared by the page's
  // four fragments) and its place in the page (the instruction's immediate offset).
  __device__ __forceinline__ bf16x8 operator()(int b, int t, int kk) const {
    const int f = (b * nib + t) * 2 + kk;
    return __builtin_bit_cast(bf16x8,
                              __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff + (f & 3) * 1024, soff + (f >> 2) * 4096, 0));
  }
};

// The forward pass of k_train_rows: the hidden layers as one software pipeline
// (weight fragments PF steps ahead, the epilogue of a block pair deferred behind
// the next pair's first products); each block pair's ReLU outputs go to LDS rows
// (layers 0..H-2) right after their epilogue; the last layer's stay in Hl.
template <int H>
__device__ __forceinline__ void forward_rows(const WBuf (&wf)[H], const uint32_t (&X0)[4][8], uint32_t (&Hl)[4][8],
                                             char* hrows, const float* sm_bias, const LaneK& K) {
  using P = PR<NVDB_BF16>;
  using CF = TrainRCfg<H>;
  constexpr int NB = 4, KS = P::KS;
  using S = FwdSteps<4, NB, H>;
  constexpr int T = S::total();
  constexpr int PF = ROWS_FWD_PF;
  P::Frag fa[PF], fb[PF];
  floatx16 acc[2][2];
  uint32_t Hs[2][NB][8];  // outputs of layers with even / odd index
  auto fetch = [&](auto gc, P::Frag& x, P::Frag& y) {
    constexpr int g = decltype(gc)::value;
    constexpr int l = S::layer(g), ob = 2 * S::pair(g), t = S::step(g) / KS, kk = S::step(g) % KS;
    x = wf[l](ob, t, kk);
    y = wf[l](ob + 1, t, kk);
  };
  auto epilogue = [&](auto lc, auto pc, floatx16& a0, floatx16& a1) {
    constexpr int le = decltype(lc)::value, pe = decltype(pc)::value;
    uint32_t(&O)[NB][8] = (le == H - 1) ? Hl : Hs[le & 1];
    store_relu<NVDB_BF16>(a0, O[2 * pe]);
    store_relu<NVDB_BF16>(a1, O[2 * pe + 1]);
    if constexpr (le < H - 1) {
      char* rows = hrows + le * CF::LROWS;
      write_row_block(rows, K, 2 * pe, O[2 * pe]);
      write_row_block(rows, K, 2 * pe + 1, O[2 * pe + 1]);
    }
  };
  static_for<0, PF>([&](auto gc) {
    constexpr int g = decltype(gc)::value;
    if constexpr (g < T) fetch(gc, fa[g], fb[g]);
  });
  // Accumulators start from the bias of their output features, loaded from LDS as
  // soon as the previous user of the accumulator set has finished (its deferred
  // epilogue), several steps before the first product reads them.
  acc[0][0] = bias_acc(sm_bias, K, 0);
  acc[0][1] = bias_acc(sm_bias, K, 1);
  static_for<0, T>([&](auto gc) {
    constexpr int g = decltype(gc)::value;
    constexpr int l = S::layer(g), p = S::pair(g), s = S::step(g), buf = S::gpair(g) & 1;
    if constexpr (s == 0 && S::gpair(g) == 0) {
      // the second accumulator set is free from the start
      constexpr int gn = g + S::nsl(l);
      if constexpr (gn < T) {
        acc[buf ^ 1][0] = bias_acc(sm_bias + S::layer(gn) * 128, K, 2 * S::pair(gn));
        acc[buf ^ 1][1] = bias_acc(sm_bias + S::layer(gn) * 128, K, 2 * S::pair(gn) + 1);
      }
    }
    const P::Frag a0 = fa[g % PF], a1 = fb[g % PF];
    if constexpr (g + PF < T) fetch(IC<g + PF>{}, fa[g % PF], fb[g % PF]);
    P::Frag b;
    if constexpr (l == 0) b = P::sfrag(X0[s / KS], s % KS);
    else b = P::sfrag(Hs[(l - 1) & 1][s / KS], s % KS);
    acc[buf][0] = P::mma(a0, b, acc[buf][0]);
    acc[buf][1] = P::mma(a1, b, acc[buf][1]);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (s == S::DEFER - 1 && S::gpair(g) > 0) {
      constexpr int ge = g - S::DEFER;  // last step of the previous pair
      if constexpr (S::deferred(ge)) epilogue(IC<S::layer(ge)>{}, IC<S::pair(ge)>{}, acc[buf ^ 1][0], acc[buf ^ 1][1]);
      // the set just released serves the pair after this one
      constexpr int gn = g - s + S::nsl(l);  // first step of the next pair
      if constexpr (gn < T) {
        acc[buf ^ 1][0] = bias_acc(sm_bias + S::layer(gn) * 128, K, 2 * S::pair(gn));
        acc[buf ^ 1][1] = bias_acc(sm_bias + S::layer(gn) * 128, K, 2 * S::pair(gn) + 1);
      }
    }
    if constexpr (s == S::nsl(l) - 1 && !S::deferred(g)) epilogue(IC<l>{}, IC<p>{}, acc[buf][0], acc[buf][1]);
  });
}

// The four products of one weight-gradient step, d_ab += A_a B_b (2 x 2 blocks of
// 32 x 32, k = 16 samples), accumulated in the accumulation registers.  The
// leading s_nop gives the two wait states a matrix product needs after a
// vector-ALU write of its operands, which the compiler does not track through
// inline assembly.
__device__ __forceinline__ void mfma_dw4(floatx16& d00, floatx16& d01, floatx16& d10, floatx16& d11, bf16x8 a0,
                                         bf16x8 a1, bf16x8 b0, bf16x8 b1) {
  asm("s_nop 1\n\t"
      "v_mfma_f32_32x32x16_bf16 %0, %4, %6, %0\n\t"
      "v_mfma_f32_32x32x16_bf16 %1, %4, %7, %1\n\t"
      "v_mfma_f32_32x32x16_bf16 %2, %5, %6, %2\n\t"
      "v_mfma_f32_32x32x16_bf16 %3, %5, %7, %3"
      : "+a"(d00), "+a"(d01), "+a"(d10), "+a"(d11)
      : "v"(a0), "v"(a1), "v"(b0), "v"(b1));
}

template <int H>
__global__ void __launch_bounds__(256, 1) __attribute__((amdgpu_waves_per_eu(1, 1))) k_train_rows(TrainLaunch L) {
  using P = PR<NVDB_BF16>;
  using CF = TrainRCfg<H>;
  constexpr int W = CF::W, NB = CF::NB, KP = CF::KP, NIB0 = CF::NIB0;
  __shared__ __attribute__((aligned(16))) char smem[CF::LDS_BYTES];

  const TrainNet& TN = L.nets[blockIdx.y];
  if (TN.prev_loss && *TN.prev_loss < *TN.stop_below) return;  // uniform: this network has converged
  const NetView& nv = TN.net;
  const SampleSpec& sp = TN.spec;
  const int wave = wave_id();
  const int wo = wave >> 1, wi = wave & 1;

  char* const hrows0 = smem;
  char* const grows0 = smem + CF::G_OFF;
  float* const gy0 = (float*)(smem + CF::GY_OFF);
  float* const sm_bias0 = (float*)(smem + CF::SMALL_OFF);  // [H][W]
  float* const sm_whead0 = sm_bias0 + H * W;               // [W]
  float* const sm_bhead0 = sm_whead0 + W;                  // [1] (padded to 4)
  float* const sm_benc0 = sm_bhead0 + 4;                   // [KP/2][4]
  float* const sm_red = sm_benc0 + 4 * (KP / 2);           // [8]
  for (int i = threadIdx.x; i < H * W; i += blockDim.x) sm_bias0[i] = nv.bias[i];
  for (int i = threadIdx.x; i < W; i += blockDim.x) sm_whead0[i] = nv.whead[i];
  if (threadIdx.x == 0) sm_bhead0[0] = nv.bhead[0];
  for (int i = threadIdx.x; i < 4 * (KP / 2); i += blockDim.x) sm_benc0[i] = nv.benc[i];
  __syncthreads();

  floatx16 dacc[H][2][2];
#pragma unroll
  for (int l = 0; l < H; ++l)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) dacc[l][a][b] = floatx16{};
  float dbias[H][1];  // bias gradient of output block 2 wo + wi
#pragma unroll
  for (int l = 0; l < H; ++l) dbias[l][0] = 0.f;
  float dwh = 0.f, dbh = 0.f, loss_acc = 0.f;

  const int64_t n_iter = (sp.n + 127) / 128;
  float* partial = TN.partial + (size_t)blockIdx.x * nv.s.pstride();
  const __amdgpu_buffer_rsrc_t wf_rsrc = raw_rsrc(nv.wfrag, wfrag_elems(nv.s) * 2);
  const __amdgpu_buffer_rsrc_t wt_rsrc = raw_rsrc(nv.wtfrag, wtfrag_elems(nv.s) * 2);
  NextSample nx{};
  {
    const int64_t j0 = (int64_t)blockIdx.x * 128 + wave * 32 + (lane_id() & 31);
    next_stage1<true>(TN, TN.tree, j0, nx);
    next_stage2<true>(TN, TN.tree, j0, nx);
  }
  for (int64_t it = blockIdx.x; it < n_iter; it += L.G) {
    const NextSample cur = nx;
    const int64_t jn = (it + L.G) * 128 + wave * 32 + (lane_id() & 31);
    next_stage1<true>(TN, TN.tree, jn, nx);
    const LaneK K = lane_consts();
    const int h = K.h, fl = K.fl;
    const int z = opaque_zero();
    const float* sm_bias = sm_bias0 + z;
    const float* sm_whead = sm_whead0 + z;
    char* hrows = hrows0 + z;
    char* grows = grows0 + z;
    float* gyl = gy0 + z;
    const int vo = lane_id() * 16;
    const int64_t j = it * 128 + wave * 32 + fl;
    Smp smp;
    smp.valid = j < sp.n;
    next_sample<true>(TN, cur, smp);

    // ================= forward: rows of a_1 .. a_{H-1} to LDS, a_H in registers
    uint32_t Hl[NB][8];
    {
      // the encoding's frequency rows are read from LDS where they are used (held in
      // registers across the iteration they would be spilled)
      PhaseA<NIB0> pa;
      pa.load(sm_benc0 + z);
      uint32_t X0[NIB0][8];
      encode_bf16_mfma<NIB0>(pa, smp, X0);
      WBuf wf[H];
#pragma unroll
      for (int l = 0; l < H; ++l)
        wf[l] = WBuf{wf_rsrc, z + (l == 0 ? 0 : (W * KP + (l - 1) * W * W) * 2), vo, l == 0 ? NIB0 : NB};
      forward_rows<H>(wf, X0, Hl, hrows + wave * CF::ROWS, sm_bias, K);
    }
    next_stage2<true>(TN, TN.tree, jn, nx);  // the next tile's leaf origin (voxels)

    // ================= head (VALU): y = Wh a_H + bh, loss, g_H = Wh^T gy * 1[a_H > 0]
    float y[1], gy[1];
    {
      float acc = 0.f;
#pragma unroll
      for (int ob = 0; ob < NB; ++ob)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const floatx4 w4 = *(const floatx4*)(sm_whead + 32 * ob + 8 * q + 4 * h);
#pragma unroll
          for (int e = 0; e < 4; ++e) acc = fmaf(w4[e], sval<NVDB_BF16>(Hl[ob], 4 * q + e), acc);
        }
      y[0] = acc + shfl_xor32(acc) + sm_bhead0[z];
    }
    const float Ls = loss_grad<1>(sp, smp, j, y, gy);
    if (h == 0) loss_acc += Ls;
    dbh += gy[0];  // per lane; both halves hold the same sample, half 0 is summed at the end
    uint32_t Gc[NB][8];
#pragma unroll
    for (int ob = 0; ob < NB; ++ob) {
      floatx16 g;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const floatx4 w4 = *(const floatx4*)(sm_whead + 32 * ob + 8 * q + 4 * h);
#pragma unroll
        for (int e = 0; e < 4; ++e) g[4 * q + e] = w4[e] * gy[0];
      }
      store_masked<NVDB_BF16>(g, Gc[ob], Hl[ob]);
    }

    // Transposed weight fragments of the input-gradient products run as one pipeline
    // over the backward stages: the first ones of a stage are requested during the
    // stage before it (those of layer H-1 before its stage's barrier), so no stage
    // starts on a load.
    constexpr int DPF = ROWS_DX_PF;
    static_assert(16 % DPF == 0, "step q of every stage uses slot q mod DPF");
    bf16x8 dfa[DPF], dfb[DPF];
    // step q = 0..15 of layer l: input blocks 2p, 2p+1 (p = q / 8), k-step q % 8 of g_l
    auto dxfetch = [&](int l, int q, bf16x8& x, bf16x8& y2) {
      const WBuf wt{wt_rsrc, z + (l - 1) * W * W * 2, vo, NB};
      const int pp = q >> 3, ss = q & 7;
      x = wt(2 * pp, ss >> 1, ss & 1);
      y2 = wt(2 * pp + 1, ss >> 1, ss & 1);
    };

    // ================= head weight gradient: a_H rows and gy of the work-group's samples
    {
      char* own = grows + wave * CF::ROWS;
#pragma unroll
      for (int t = 0; t < NB; ++t) write_row_block(own, K, t, Hl[t]);
      if (h == 0) gyl[wave * 32 + fl] = gy[0];
      __syncthreads();
      // wave w owns the head's input block w
#pragma unroll
      for (int sl = 0; sl < 4; ++sl)
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
          const bf16x8 hh = frag_tr(grows + sl * CF::ROWS, K, 16 * kk, wave);
          const u32x4 u = __builtin_bit_cast(u32x4, hh);
          const floatx4 g0 = *(const floatx4*)(gyl + sl * 32 + 16 * kk + 4 * h);
          const floatx4 g1 = *(const floatx4*)(gyl + sl * 32 + 16 * kk + 8 + 4 * h);
          dwh = fmaf(g0[0], bf16_lo(u[0]), dwh);
          dwh = fmaf(g0[1], bf16_hi(u[0]), dwh);
          dwh = fmaf(g0[2], bf16_lo(u[1]), dwh);
          dwh = fmaf(g0[3], bf16_hi(u[1]), dwh);
          dwh = fmaf(g1[0], bf16_lo(u[2]), dwh);
          dwh = fmaf(g1[1], bf16_hi(u[2]), dwh);
          dwh = fmaf(g1[2], bf16_lo(u[3]), dwh);
          dwh = fmaf(g1[3], bf16_hi(u[3]), dwh);
        }
      __syncthreads();
    }

    // ================= backward stages, layer H-1 down to 0
    static_for<0, H>([&](auto kc) {
      constexpr int l = H - 1 - decltype(kc)::value;
      // input activations of layer l as rows: a_l, or gamma recomputed into the rows of
      // a_{H-1}, which were last read by the first stage
      char* arows = hrows + (l == 0 ? H - 2 : l - 1) * CF::LROWS;
      write_rows_bf16<NB>(grows + wave * CF::ROWS, K, Gc);
      if constexpr (l == 0) {
        PhaseA<NIB0> pa;
        pa.load(sm_benc0 + z);
        uint32_t X0[NIB0][8];
        encode_bf16_mfma<NIB0>(pa, smp, X0);
        write_rows_bf16<NIB0>(arows + wave * CF::ROWS, K, X0);
      }
      if constexpr (l == H - 1) {
#pragma unroll
        for (int q = 0; q < DPF; ++q) dxfetch(H - 1, q, dfa[q], dfb[q]);
      }
      __syncthreads();
      // dW_l: 8 steps (slot sl of the four waves' rows, k-step kk of its 32 samples),
      // 2 x 2 blocks each; interleaved with the input-gradient products of l > 0:
      // Gn = (W_l^T g_l) * 1[a_l > 0], two block pairs of 8 steps
      constexpr int NDW = 8;
      bf16x8 ga[2][2], hb[2][2];
      // A[0] is the wave's own output block 2 wo + wi (whose bias gradient it sums),
      // A[1] the other block of the pair
      auto dw_load = [&](int st, bf16x8 (&A)[2], bf16x8 (&Bv)[2]) {
        const int sl = st >> 1, kk = st & 1;
        A[0] = frag_tr(grows + sl * CF::ROWS, K, 16 * kk, 2 * wo + wi);
        A[1] = frag_tr(grows + sl * CF::ROWS, K, 16 * kk, 2 * wo + (wi ^ 1));
        Bv[0] = frag_tr(arows + sl * CF::ROWS, K, 16 * kk, 2 * wi);
        Bv[1] = frag_tr(arows + sl * CF::ROWS, K, 16 * kk, 2 * wi + 1);
      };
      auto dw_step = [&](const bf16x8 (&A)[2], const bf16x8 (&Bv)[2]) {
        dbias[l][0] = frag_sum(A[0], dbias[l][0]);
        mfma_dw4(dacc[l][0][0], dacc[l][0][1], dacc[l][1][0], dacc[l][1][1], A[0], A[1], Bv[0], Bv[1]);
      };
      dw_load(0, ga[0], hb[0]);
      if constexpr (l > 0) {
        const char* own_a = arows + wave * CF::ROWS;
        uint32_t Gn[NB][8];
        floatx16 a0 = floatx16{}, a1 = floatx16{};
        uint32_t m0[8], m1[8];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int pp = q >> 3, ss = q & 7;
          const bf16x8 w0 = dfa[q % DPF], w1 = dfb[q % DPF];
          if (q + DPF < 16) dxfetch(l, q + DPF, dfa[q % DPF], dfb[q % DPF]);
          else if (l > 1) dxfetch(l - 1, q + DPF - 16, dfa[q % DPF], dfb[q % DPF]);  // the next stage's first
          const bf16x8 bg = P::sfrag(Gc[ss >> 1], ss & 1);
          a0 = P::mma(w0, bg, a0);
          a1 = P::mma(w1, bg, a1);
          if (q & 1) {
            const int st = q >> 1;
            if (st + 1 < NDW) dw_load(st + 1, ga[(st + 1) & 1], hb[(st + 1) & 1]);
            dw_step(ga[st & 1], hb[st & 1]);
          }
          __builtin_amdgcn_sched_barrier(0);
          if (ss == 1) {  // the ReLU-derivative source of this pair, six steps ahead (measured best)
            read_row_block(own_a, K, 2 * pp, m0);
            read_row_block(own_a, K, 2 * pp + 1, m1);
          }
          if (ss == 7) {
            store_masked<NVDB_BF16>(a0, Gn[2 * pp], m0);
            store_masked<NVDB_BF16>(a1, Gn[2 * pp + 1], m1);
            a0 = floatx16{};
            a1 = floatx16{};
          }
        }
#pragma unroll
        for (int ib = 0; ib < NB; ++ib)
#pragma unroll
          for (int q = 0; q < 8; ++q) Gc[ib][q] = Gn[ib][q];
      } else {
#pragma unroll
        for (int st = 0; st < NDW; ++st) {
          if (st + 1 < NDW) dw_load(st + 1, ga[(st + 1) & 1], hb[(st + 1) & 1]);
          dw_step(ga[st & 1], hb[st & 1]);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      __syncthreads();
    });
  }

  // ---- this work-group's partial gradient row; the wait states let the last
  // weight-gradient products (hidden from the compiler's hazard tracking) finish
  // before their registers are read
  asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7\n\ts_nop 7");
  const int h = lane_id() >> 5, fl = lane_id() & 31;
#pragma unroll
  for (int l = 0; l < H; ++l) {
    const int win = nv.s.win(l);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int ob = 2 * wo + (a ^ wi), ib = 2 * wi + b, i = 32 * ib + fl;
        if (i < win) {
#pragma unroll
          for (int r = 0; r < 16; ++r) partial[nv.s.woff(l) + (size_t)sfeat(ob, r, h) * win + i] = dacc[l][a][b][r];
        }
      }
  }
  // biases: wave (wo, wi) owns output block 2 wo + wi; lane halves combined
#pragma unroll
  for (int l = 0; l < H; ++l) {
    const float v = dbias[l][0] + shfl_xor32(dbias[l][0]);
    if (h == 0) partial[nv.s.boff(l) + 32 * (2 * wo + wi) + fl] = v;
  }
  {
    const float v = dwh + shfl_xor32(dwh);
    if (h == 0) partial[nv.s.woff(H) + 32 * wave + fl] = v;
  }
  // head bias and loss: fixed-order reductions over each wave's half 0, then over the waves
  float v = loss_acc, vb = (h == 0) ? dbh : 0.f;
#pragma unroll
  for (int off = 16; off >= 1; off >>= 1) {
    int src = (lane_id() ^ off) << 2;
    v += __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v)));
    vb += __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(vb)));
  }
  if (lane_id() == 0) {
    sm_red[wave] = v;
    sm_red[4 + wave] = vb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    TN.loss_partial[blockIdx.x] = ((sm_red[0] + sm_red[1]) + sm_red[2]) + sm_red[3];
    partial[nv.s.boff(H)] = ((sm_red[4] + sm_red[5]) + sm_red[6]) + sm_red[7];
  }
}

void (*train_rows_kernel(int H))(TrainLaunch) {
  if (H == 4) return k_train_rows<4>;
  if (H == 3) return k_train_rows<3>;
  return nullptr;
}

}  // namespace nvdb
