// C-ABI of libnvdb: argument checking, object lifetime and launch sequencing.
// The arithmetic lives in mlp.hip (networks) and tree.hip (tree build, errors).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <cfloat>
#include <limits>
#include <map>
#include <mutex>
#include <memory>
#include <new>
#include <string>

#include "nvdb_internal.h"

namespace nvdb {

constexpr int MAX_G = 512;        // work-groups (partial gradient rows) per network
constexpr int DEFAULT_G = 256;    // used until nvdb_autotune picks another
constexpr int TRAIN_TILE = 128;   // samples per work-group iteration

struct Net {
  bool present = false;
  nvdb_net_desc d{};
  NetShape s{};
  KernelSet ks{};
  int prec = NVDB_BF16;
  DevBuf<float> theta, m, v, grad;
  DevBuf<float> partial, loss_partial, losses;
  DevBuf<int32_t> ran;  // per step of a sequence fit: 1 when the step ran
  DevBuf<floatx4> xt;  // gathered samples of the current step
  DevBuf<char> wrow, wcol, wfrag, wtfrag;
  // FP8 form: e4m3 fragments and per-layer scales, rebuilt from theta by every FP8 decode
  mutable DevBuf<char> w8;
  mutable DevBuf<float> w8inv;
  DevBuf<float> bias, whead, bhead, benc;
  // workspace of the _dev calls (nvdb_model_reserve_dev): fixed addresses, so
  // graphs that record those calls stay valid until the next reservation
  DevBuf<float> dpart, dlossp;
  DevBuf<floatx4> dxt;
  int64_t dev_n = 0;
  int dev_G = 0;
  int64_t step = 0;
  bool params_set = false, enc_set = false;
};

}  // namespace nvdb

struct nvdb_tree : nvdb::Tree {};
struct nvdb_model {
  nvdb_model_desc d{};
  nvdb::Net nets[NVDB_MAX_NETS];
  int train_g = 0;  // work-groups per network chosen by nvdb_autotune (0: default)
  // recorded on the caller's stream after the model's enqueued work; host-side
  // parameter copies wait for it instead of the whole device
  hipEvent_t done = nullptr;
  // [0]: explicit sample indices found at or beyond their population size
  nvdb::DevBuf<unsigned long long> errw;
  // events of the optional per-launch timing of nvdb_fit, created once and reused
  // (creating thousands per call would leave the device idle before every fit)
  std::vector<hipEvent_t> timing;
  ~nvdb_model() {
    if (done) (void)hipEventDestroy(done);
    for (auto e : timing) (void)hipEventDestroy(e);
  }
};

using namespace nvdb;

static thread_local std::string g_err;

template <class F>
static nvdb_status guarded(F&& f) {
  try {
    f();
    g_err.clear();
    return NVDB_OK;
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return NVDB_E_NOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return NVDB_E_INVALID;
  } catch (...) {
    g_err = "unknown error";
    return NVDB_E_INVALID;
  }
}

static TreeView tree_view(const Tree* t) {
  TreeView v{};
  if (!t) return v;
  v.leaf_o = t->leaf_o.p;
  v.leaf_mask = t->leaf_mask.p;
  v.vox_key = t->vox_key.p;
  v.tile_key = t->tile_key.p;
  v.tile_val = t->tile_val.p;
  v.values = t->values.p;
  v.l1_o = t->l1_o.p;
  v.l1_child = t->l1_child.p;
  v.l1_active = t->l1_active.p;
  return v;
}

static NetView net_view(const Net& n) {
  NetView v{};
  v.s = n.s;
  v.wrow = n.wrow.p;
  v.wcol = n.wcol.p;
  v.wfrag = n.wfrag.p;
  v.wtfrag = n.wtfrag.p;
  v.bias = n.bias.p;
  v.whead = n.whead.p;
  v.bhead = n.bhead.p;
  v.benc = n.benc.p;
  v.nfreq = n.d.n_freq;
  v.act_w = n.d.sin_freq;
  v.act_rev64 = (double)n.d.sin_freq / (2.0 * 3.14159265358979323846);
  v.act_rev = (float)v.act_rev64;
  return v;
}

static AdamNet adam_view(Net& n) {
  AdamNet a{};
  a.s = n.s;
  a.theta = n.theta.p;
  a.m = n.m.p;
  a.v = n.v.p;
  a.prec = n.prec;
  a.wrow = n.wrow.p;
  a.wcol = n.wcol.p;
  a.wfrag = n.wfrag.p;
  a.wtfrag = n.wtfrag.p;
  a.bias = n.bias.p;
  a.whead = n.whead.p;
  a.bhead = n.bhead.p;
  return a;
}

static void base_spec(const nvdb_model* m, SampleSpec* sp) {
  std::memset(sp, 0, sizeof(*sp));
  for (int d = 0; d < 3; ++d) sp->lo[d] = m->d.domain_lo[d];
  sp->inv_d = 1.f / (float)m->d.domain_size;
  sp->tscale = 1.f / m->d.value_scale;
}

static Net& net_of(nvdb_model* m, int32_t net) {
  NVDB_REQUIRE(m != nullptr, NVDB_E_INVALID, "model is null");
  NVDB_REQUIRE(net >= 0 && net < NVDB_MAX_NETS && m->nets[net].present, NVDB_E_INVALID, "network not in model");
  return m->nets[net];
}
static const Net& net_of(const nvdb_model* m, int32_t net) { return net_of(const_cast<nvdb_model*>(m), net); }

// The model's work enqueued on `st` so far: host copies of its state wait for this.
// Not recorded while `st` is being captured into a graph: the graph's launch is the
// caller's to order.
static void mark(const nvdb_model* m, hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  NVDB_HIP(hipStreamIsCapturing(st, &cs));
  if (cs == hipStreamCaptureStatusNone) NVDB_HIP(hipEventRecord(m->done, st));
}
static void wait_model(const nvdb_model* m) { NVDB_HIP(hipEventSynchronize(m->done)); }

// Reads and clears the model's count of out-of-range sample indices (waits for its work).
static int64_t take_bad_indices(const nvdb_model* m) {
  wait_model(m);
  unsigned long long v = 0;
  NVDB_HIP(hipMemcpy(&v, m->errw.p, sizeof(v), hipMemcpyDeviceToHost));
  if (v) NVDB_HIP(hipMemset(m->errw.p, 0, sizeof(v)));
  return (int64_t)v;
}

static void ensure_partials(Net& n, int G) {
  n.partial.ensure((size_t)G * n.s.pstride());
  n.loss_partial.ensure(G);
}

extern "C" {

const char* nvdb_last_error(void) { return g_err.c_str(); }
int32_t nvdb_abi_version(void) { return 2; }

// ------------------------------------------------------------------ trees
nvdb_status nvdb_tree_build_dense(const float* grid_dev, const int32_t dims[3], const int32_t origin[3],
                                  const nvdb_active_rule* rule, void* stream, nvdb_tree** out) {
  return guarded([&] {
    NVDB_REQUIRE(out && dims && origin && rule, NVDB_E_INVALID, "null argument");
    *out = nullptr;
    Tree* t = build_tree_dense(grid_dev, dims, origin, *rule, (hipStream_t)stream);
    *out = static_cast<nvdb_tree*>(t);
  });
}

nvdb_status nvdb_tree_build_sparse(const int32_t* ijk_dev, const float* values_dev, int64_t n,
                                   const nvdb_active_rule* rule, void* stream, nvdb_tree** out) {
  return guarded([&] {
    NVDB_REQUIRE(out && rule, NVDB_E_INVALID, "null argument");
    *out = nullptr;
    Tree* t = build_tree_sparse(ijk_dev, values_dev, n, *rule, (hipStream_t)stream);
    *out = static_cast<nvdb_tree*>(t);
  });
}

nvdb_status nvdb_tree_get_info(const nvdb_tree* t, nvdb_tree_info* info) {
  return guarded([&] {
    NVDB_REQUIRE(t && info, NVDB_E_INVALID, "null argument");
    std::memset(info, 0, sizeof(*info));
    info->n_voxels = t->n_vox;
    info->n_leaves = t->n_leaf;
    info->n_l1 = t->n_l1;
    info->n_l2 = t->n_l2;
    for (int d = 0; d < 3; ++d) {
      info->grid_origin[d] = t->origin[d];
      info->grid_dims[d] = t->dims[d];
    }
    // Tab. memory_cost accounting of the explicit tree
    info->bytes_l2 = t->n_l2 * (2 * (32768 / 8) + 32768 * 1 + 12);
    info->bytes_l1 = t->n_l1 * (2 * (4096 / 8) + 4096 * 4 + 12);
    info->bytes_leaf_masks = t->n_leaf * (512 / 8 + 12);
    info->bytes_voxels = t->n_leaf * 512 * 4;
    info->n_tiles = t->n_tile;
  });
}

nvdb_status nvdb_tree_prune_tiles(const nvdb_tree* in, void* stream, nvdb_tree** out) {
  return guarded([&] {
    NVDB_REQUIRE(in && out, NVDB_E_INVALID, "null argument");
    *out = nullptr;
    Tree* t = prune_tiles(*in, (hipStream_t)stream);
    *out = static_cast<nvdb_tree*>(t);
  });
}

nvdb_status nvdb_tree_export_tiles(const nvdb_tree* t, uint32_t* tile_key, float* tile_value, uint64_t* l1_active) {
  return guarded([&] {
    NVDB_REQUIRE(t, NVDB_E_INVALID, "null tree");
    if (tile_key && t->n_tile)
      NVDB_HIP(hipMemcpy(tile_key, t->tile_key.p, t->n_tile * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (tile_value && t->n_tile)
      NVDB_HIP(hipMemcpy(tile_value, t->tile_val.p, t->n_tile * sizeof(float), hipMemcpyDeviceToHost));
    if (l1_active && t->n_l1)
      NVDB_HIP(hipMemcpy(l1_active, t->l1_active.p, t->n_l1 * 64 * sizeof(uint64_t), hipMemcpyDeviceToHost));
  });
}

nvdb_status nvdb_tree_export(const nvdb_tree* t, int32_t* leaf_origin, uint64_t* leaf_mask, uint32_t* leaf_off,
                             float* values, int32_t* l1_origin, uint64_t* l1_child) {
  return guarded([&] {
    NVDB_REQUIRE(t, NVDB_E_INVALID, "null tree");
    if (leaf_origin && t->n_leaf) {
      std::vector<int4> o(t->n_leaf);
      NVDB_HIP(hipMemcpy(o.data(), t->leaf_o.p, t->n_leaf * sizeof(int4), hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < t->n_leaf; ++i) {
        leaf_origin[3 * i] = o[i].x;
        leaf_origin[3 * i + 1] = o[i].y;
        leaf_origin[3 * i + 2] = o[i].z;
      }
    }
    if (leaf_mask && t->n_leaf)
      NVDB_HIP(hipMemcpy(leaf_mask, t->leaf_mask.p, t->n_leaf * 8 * sizeof(uint64_t), hipMemcpyDeviceToHost));
    if (leaf_off) NVDB_HIP(hipMemcpy(leaf_off, t->leaf_off.p, (t->n_leaf + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (values && t->n_vox) NVDB_HIP(hipMemcpy(values, t->values.p, t->n_vox * sizeof(float), hipMemcpyDeviceToHost));
    if (l1_origin && t->n_l1) {
      std::vector<int4> o(t->n_l1);
      NVDB_HIP(hipMemcpy(o.data(), t->l1_o.p, t->n_l1 * sizeof(int4), hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < t->n_l1; ++i) {
        l1_origin[3 * i] = o[i].x;
        l1_origin[3 * i + 1] = o[i].y;
        l1_origin[3 * i + 2] = o[i].z;
      }
    }
    if (l1_child && t->n_l1)
      NVDB_HIP(hipMemcpy(l1_child, t->l1_child.p, t->n_l1 * 64 * sizeof(uint64_t), hipMemcpyDeviceToHost));
  });
}

nvdb_status nvdb_tree_export_l2(const nvdb_tree* t, int32_t* l2_origin, uint64_t* l2_child) {
  return guarded([&] {
    NVDB_REQUIRE(t, NVDB_E_INVALID, "null tree");
    if (l2_origin && t->n_l2) std::memcpy(l2_origin, t->l2_origin.data(), t->n_l2 * 3 * sizeof(int32_t));
    if (l2_child && t->n_l2) {
      std::memset(l2_child, 0, t->n_l2 * 512 * sizeof(uint64_t));
      std::vector<int4> o(t->n_l1);
      if (t->n_l1) NVDB_HIP(hipMemcpy(o.data(), t->l1_o.p, t->n_l1 * sizeof(int4), hipMemcpyDeviceToHost));
      int64_t node = -1;
      int32_t cur[3] = {0, 0, 0};
      for (const int4& q : o) {  // level-1 nodes are grouped by level-2 node, in canonical order
        const int32_t l2[3] = {q.x & ~4095, q.y & ~4095, q.z & ~4095};
        if (node < 0 || l2[0] != cur[0] || l2[1] != cur[1] || l2[2] != cur[2]) {
          ++node;
          std::memcpy(cur, l2, sizeof(cur));
        }
        NVDB_REQUIRE(node < t->n_l2, NVDB_E_STATE, "level-1 nodes out of canonical order");
        const int n2 = (((q.x >> 7) & 31) << 10) | (((q.y >> 7) & 31) << 5) | ((q.z >> 7) & 31);
        l2_child[node * 512 + (n2 >> 6)] |= 1ull << (n2 & 63);
      }
    }
  });
}

void nvdb_tree_free(nvdb_tree* t) { delete t; }

// ------------------------------------------------------------------ models
nvdb_status nvdb_model_create(const nvdb_model_desc* desc, nvdb_model** out) {
  return guarded([&] {
    NVDB_REQUIRE(desc && out, NVDB_E_INVALID, "null argument");
    *out = nullptr;
    NVDB_REQUIRE(desc->precision == NVDB_FP32 || desc->precision == NVDB_BF16, NVDB_E_INVALID, "unknown precision");
    NVDB_REQUIRE(desc->domain_size > 0, NVDB_E_INVALID, "domain_size must be positive");
    NVDB_REQUIRE(std::isfinite(desc->value_scale) && desc->value_scale > 0.f, NVDB_E_INVALID,
                 "value_scale must be positive");
    nvdb_model* m = new nvdb_model();
    try {
      m->d = *desc;
      bool any = false;
      for (int k = 0; k < NVDB_MAX_NETS; ++k) {
        if (!desc->has_net[k]) continue;
        any = true;
        Net& n = m->nets[k];
        const nvdb_net_desc& d = desc->net[k];
        NVDB_REQUIRE(d.n_freq > 0 && 2 * d.n_freq <= 256, NVDB_E_UNSUPPORTED, "n_freq must be in 1..128");
        NVDB_REQUIRE(d.n_out == 1 || d.n_out == 3, NVDB_E_UNSUPPORTED, "n_out must be 1 or 3");
        NVDB_REQUIRE(k != NVDB_NET_L1 || d.n_out == 3, NVDB_E_INVALID, "the level-1 classifier has 3 outputs");
        NVDB_REQUIRE(k == NVDB_NET_L1 || d.n_out == 1, NVDB_E_INVALID, "regressor and level-0 classifier have 1 output");
        n.present = true;
        n.d = d;
        n.prec = desc->precision;
        n.s.K = 2 * d.n_freq;
        n.s.KP = std::max(64, ((n.s.K + 31) / 32) * 32);
        n.s.W = d.width;
        n.s.H = d.hidden;
        n.s.C = d.n_out;
        NVDB_REQUIRE(std::isfinite(d.sin_freq) && d.sin_freq >= 0.f && d.sin_freq <= 64.f, NVDB_E_INVALID,
                     "sin frequency must be 0 (ReLU) or in (0, 64]");
        const int act = d.sin_freq > 0.f ? ACT_SIN : ACT_RELU;
        NVDB_REQUIRE(find_kernels(n.prec, d.width, d.hidden, n.s.KP, d.n_out, act, &n.ks), NVDB_E_UNSUPPORTED,
                     "no kernel for this network shape (width " + std::to_string(d.width) + ", hidden " +
                         std::to_string(d.hidden) + ", inputs " + std::to_string(n.s.KP) + ", outputs " +
                         std::to_string(d.n_out) + (act == ACT_SIN ? ", sin activation" : "") + ")");
        if (n.prec == NVDB_BF16 && d.n_freq == 64 && n.ks.train_rows && !std::getenv("NVDB_TRAIN_CLASSIC"))
          n.ks.train = n.ks.train_rows;
        const int64_t P = n.s.nparams();
        n.theta.alloc(P);
        n.m.alloc(P);
        n.v.alloc(P);
        n.grad.alloc(P);
        NVDB_HIP(hipMemset(n.m.p, 0, P * 4));
        NVDB_HIP(hipMemset(n.v.p, 0, P * 4));
        const int W = n.s.W, H = n.s.H, KP = n.s.KP;
        if (n.prec == NVDB_BF16) {
          n.wrow.alloc((size_t)H * W * ROW_ELEMS * 2);
          n.wfrag.alloc((size_t)wfrag_elems(n.s) * 2);
          n.wtfrag.alloc((size_t)std::max<int64_t>(1, wtfrag_elems(n.s)) * 2);
          NVDB_HIP(hipMemset(n.wrow.p, 0, n.wrow.n));
          NVDB_HIP(hipMemset(n.wfrag.p, 0, n.wfrag.n));
          NVDB_HIP(hipMemset(n.wtfrag.p, 0, n.wtfrag.n));
        } else {
          const size_t elems = (size_t)KP * W + (size_t)(H - 1) * W * W;
          n.wrow.alloc(elems * 4);
          n.wcol.alloc(elems * 4);
          NVDB_HIP(hipMemset(n.wrow.p, 0, n.wrow.n));
          NVDB_HIP(hipMemset(n.wcol.p, 0, n.wcol.n));
        }
        n.bias.alloc((size_t)H * W);
        n.whead.alloc((size_t)n.s.C * W);
        n.bhead.alloc(4);
        n.benc.alloc((size_t)4 * (KP / 2));
        NVDB_HIP(hipMemset(n.bhead.p, 0, 16));
        NVDB_HIP(hipMemset(n.benc.p, 0, n.benc.n * 4));
      }
      NVDB_REQUIRE(any, NVDB_E_INVALID, "model has no networks");
      NVDB_HIP(hipEventCreateWithFlags(&m->done, hipEventDisableTiming));
      m->errw.alloc(1);
      NVDB_HIP(hipMemset(m->errw.p, 0, sizeof(unsigned long long)));
    } catch (...) {
      delete m;
      throw;
    }
    *out = m;
  });
}

nvdb_status nvdb_model_param_count(const nvdb_model* m, int32_t net, int64_t* n) {
  return guarded([&] {
    NVDB_REQUIRE(n, NVDB_E_INVALID, "null argument");
    *n = net_of(m, net).s.nparams();
  });
}

nvdb_status nvdb_model_set_params(nvdb_model* m, int32_t net, const float* params, int64_t n) {
  return guarded([&] {
    Net& N = net_of(m, net);
    NVDB_REQUIRE(params && n == N.s.nparams(), NVDB_E_INVALID, "parameter count mismatch");
    for (int64_t i = 0; i < n; ++i) NVDB_REQUIRE(std::isfinite(params[i]), NVDB_E_INVALID, "non-finite parameter");
    wait_model(m);
    NVDB_HIP(hipMemcpy(N.theta.p, params, n * 4, hipMemcpyHostToDevice));
    launch_write_shadow(adam_view(N), nullptr);
    NVDB_HIP(hipStreamSynchronize(nullptr));
    N.params_set = true;
  });
}

nvdb_status nvdb_model_get_params(const nvdb_model* m, int32_t net, float* params, int64_t n) {
  return guarded([&] {
    const Net& N = net_of(m, net);
    NVDB_REQUIRE(params && n == N.s.nparams(), NVDB_E_INVALID, "parameter count mismatch");
    wait_model(m);
    NVDB_HIP(hipMemcpy(params, N.theta.p, n * 4, hipMemcpyDeviceToHost));
  });
}

// ---------------------------------------------------------------- 16-bit storage
// float32 -> IEEE binary16, round to nearest even (overflow to infinity, NaN kept).
static uint16_t f32_to_f16(float f) {
  uint32_t x;
  std::memcpy(&x, &f, 4);
  const uint32_t sign = (x >> 16) & 0x8000u;
  const uint32_t ax = x & 0x7fffffffu;
  if (ax >= 0x7f800000u) return (uint16_t)(sign | 0x7c00u | (ax > 0x7f800000u ? 0x200u : 0u));  // inf / NaN
  const int e = (int)(ax >> 23) - 127;  // unbiased exponent
  if (e > 15) return (uint16_t)(sign | 0x7c00u);
  uint32_t mant = (ax & 0x7fffffu) | 0x800000u;  // 24-bit significand (normal inputs)
  int shift;                                     // bits dropped from the 24-bit significand
  uint32_t ebits;
  if (e >= -14) {  // normal half: keep 11 bits
    shift = 13;
    ebits = (uint32_t)(e + 15) << 10;
  } else {  // subnormal half (or underflow to zero): value = m * 2^-24
    if (ax < 0x33000000u) return (uint16_t)sign;  // below half the smallest subnormal
    shift = 13 + (-14 - e);
    ebits = 0;
  }
  uint32_t q = mant >> shift;
  const uint32_t rem = mant & ((1u << shift) - 1u), half = 1u << (shift - 1);
  if (rem > half || (rem == half && (q & 1u))) ++q;  // round to nearest even
  if (ebits) {
    // q carries the implicit bit at bit 10 (bit 11 after a rounding carry); adding
    // it to the biased exponent field moves the carry into the exponent
    const uint32_t h = ebits + q - 0x400u;
    return (uint16_t)(sign | (h >= 0x7c00u ? 0x7c00u : h));
  }
  return (uint16_t)(sign | q);  // subnormal; a carry into bit 10 yields the smallest normal
}
// float32 -> bfloat16, round to nearest even (NaN kept quiet).
static uint16_t f32_to_bf16(float f) {
  uint32_t x;
  std::memcpy(&x, &f, 4);
  if ((x & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((x >> 16) | 0x40u);
  return (uint16_t)((x + 0x7fffu + ((x >> 16) & 1u)) >> 16);
}
static float f16_to_f32(uint16_t h) {
  const uint32_t sign = (uint32_t)(h & 0x8000u) << 16, e = (h >> 10) & 31u, m = h & 0x3ffu;
  float v;
  if (e == 0) v = std::ldexp((float)m, -24);
  else if (e == 31) v = m ? std::numeric_limits<float>::quiet_NaN() : std::numeric_limits<float>::infinity();
  else v = std::ldexp((float)(m | 0x400u), (int)e - 25);
  uint32_t x;
  std::memcpy(&x, &v, 4);
  x |= sign;
  std::memcpy(&v, &x, 4);
  return v;
}
static float bf16_to_f32(uint16_t b) {
  const uint32_t x = (uint32_t)b << 16;
  float v;
  std::memcpy(&v, &x, 4);
  return v;
}

nvdb_status nvdb_model_get_params16(const nvdb_model* m, int32_t net, int32_t kind, uint16_t* dst, int64_t n) {
  return guarded([&] {
    NVDB_REQUIRE(kind == NVDB_STORE_F16 || kind == NVDB_STORE_BF16, NVDB_E_INVALID, "unknown 16-bit format");
    const Net& N = net_of(m, net);
    NVDB_REQUIRE(dst && n == N.s.nparams(), NVDB_E_INVALID, "parameter count mismatch");
    std::vector<float> f((size_t)n);
    wait_model(m);
    NVDB_HIP(hipMemcpy(f.data(), N.theta.p, n * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) dst[i] = kind == NVDB_STORE_F16 ? f32_to_f16(f[i]) : f32_to_bf16(f[i]);
  });
}

nvdb_status nvdb_model_set_params16(nvdb_model* m, int32_t net, int32_t kind, const uint16_t* src, int64_t n) {
  std::vector<float> f;
  const nvdb_status st = guarded([&] {
    NVDB_REQUIRE(kind == NVDB_STORE_F16 || kind == NVDB_STORE_BF16, NVDB_E_INVALID, "unknown 16-bit format");
    NVDB_REQUIRE(src && n >= 0 && n < (1ll << 31), NVDB_E_INVALID, "bad parameters");
    f.resize((size_t)n);
    for (int64_t i = 0; i < n; ++i) f[i] = kind == NVDB_STORE_F16 ? f16_to_f32(src[i]) : bf16_to_f32(src[i]);
  });
  if (st != NVDB_OK) return st;
  return nvdb_model_set_params(m, net, f.data(), n);
}

nvdb_status nvdb_model_set_encoding(nvdb_model* m, int32_t net, const float* B, int32_t n_freq) {
  return guarded([&] {
    Net& N = net_of(m, net);
    NVDB_REQUIRE(B && n_freq == N.d.n_freq, NVDB_E_INVALID, "n_freq mismatch");
    std::vector<float> h((size_t)4 * (N.s.KP / 2), 0.f);  // rows (bx, by, bz, 0)
    for (int i = 0; i < n_freq; ++i)
      for (int d = 0; d < 3; ++d) {
        NVDB_REQUIRE(std::isfinite(B[3 * i + d]), NVDB_E_INVALID, "non-finite encoding matrix");
        h[4 * i + d] = B[3 * i + d];
      }
    NVDB_HIP(hipMemcpy(N.benc.p, h.data(), h.size() * 4, hipMemcpyHostToDevice));
    N.enc_set = true;
  });
}

nvdb_status nvdb_model_get_opt_state(const nvdb_model* m, int32_t net, float* mm, float* vv, int64_t n,
                                     int64_t* step) {
  return guarded([&] {
    const Net& N = net_of(m, net);
    NVDB_REQUIRE(n == N.s.nparams(), NVDB_E_INVALID, "parameter count mismatch");
    wait_model(m);
    if (mm) NVDB_HIP(hipMemcpy(mm, N.m.p, n * 4, hipMemcpyDeviceToHost));
    if (vv) NVDB_HIP(hipMemcpy(vv, N.v.p, n * 4, hipMemcpyDeviceToHost));
    if (step) *step = N.step;
  });
}

nvdb_status nvdb_model_set_opt_state(nvdb_model* m, int32_t net, const float* mm, const float* vv, int64_t n,
                                     int64_t step) {
  return guarded([&] {
    Net& N = net_of(m, net);
    NVDB_REQUIRE(mm && vv && n == N.s.nparams() && step >= 0, NVDB_E_INVALID, "bad optimiser state");
    wait_model(m);
    NVDB_HIP(hipMemcpy(N.m.p, mm, n * 4, hipMemcpyHostToDevice));
    NVDB_HIP(hipMemcpy(N.v.p, vv, n * 4, hipMemcpyHostToDevice));
    N.step = step;
  });
}

void nvdb_model_free(nvdb_model* m) { delete m; }

// ------------------------------------------------------------------ fit
static int population_src(int net, const Tree* t, int64_t* pop) {
  if (net == NVDB_NET_REGRESSOR) {
    *pop = t->n_vox;
    return SRC_VOXELS;
  }
  if (net == NVDB_NET_L0) {
    *pop = 512 * t->n_leaf;
    return SRC_LEAF_SLOTS;
  }
  if (net == NVDB_NET_TILE) {
    *pop = t->n_tile;
    return SRC_TILES;
  }
  *pop = 4096 * t->n_l1;
  return SRC_L1_SLOTS;
}

}  // extern "C"

// Schedule of one run of consecutive optimiser steps.
struct Phase {
  int32_t batch;
  uint64_t seed;
  float lr, lr_decay;
  int32_t lr_interval;
  const nvdb_fit_desc* idx;  // explicit index lists (idx_dev / idx_count) or null for i.i.d. draws
};

// Per-step device pointers: where each network's batch loss goes and the
// optional stop test of warm-started frames.
struct StepHooks {
  float* grad_out[NVDB_MAX_NETS] = {};  // non-null: write the summed gradient there, no Adam step
  float* loss_out[NVDB_MAX_NETS] = {};
  const float* prev_loss[NVDB_MAX_NETS] = {};
  const float* stop_below[NVDB_MAX_NETS] = {};
  int32_t* ran[NVDB_MAX_NETS] = {};
};

static int train_grid(int64_t n, int g = DEFAULT_G) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, (n + TRAIN_TILE - 1) / TRAIN_TILE));
}

// Networks that share a kernel go into one launch (gridDim.y = network).
static std::vector<std::vector<int>> kernel_groups(const nvdb_model* m, const std::vector<int>& nets) {
  std::vector<std::vector<int>> groups;
  for (int k : nets) {
    bool put = false;
    for (auto& g : groups)
      if (m->nets[g[0]].ks.train == m->nets[k].ks.train) {
        g.push_back(k);
        put = true;
        break;
      }
    if (!put) groups.push_back({k});
  }
  return groups;
}

// Checks that every selected network is ready and has a non-empty population on `tree`.
static std::vector<int> fit_nets(nvdb_model* m, const Tree* tree, int32_t mask) {
  std::vector<int> nets;
  for (int k = 0; k < NVDB_MAX_NETS; ++k) {
    if (!(mask & (1 << k))) continue;
    Net& N = net_of(m, k);
    NVDB_REQUIRE(N.params_set && N.enc_set, NVDB_E_STATE, "parameters or encoding not set");
    int64_t pop;
    population_src(k, tree, &pop);
    NVDB_REQUIRE(pop > 0 && pop < (1ll << 32), NVDB_E_INVALID, "empty or oversized population");
    nets.push_back(k);
  }
  NVDB_REQUIRE(!nets.empty(), NVDB_E_INVALID, "no network selected");
  return nets;
}

static void check_schedule(const nvdb_fit_desc* f) {
  NVDB_REQUIRE(f->steps >= 0 && f->batch >= 1 && f->batch <= (1 << 24), NVDB_E_INVALID, "bad steps/batch");
  NVDB_REQUIRE(std::isfinite(f->lr) && f->lr >= 0.f && std::isfinite(f->lr_decay) && f->lr_decay > 0.f &&
                   f->lr_interval >= 1,
               NVDB_E_INVALID, "bad learning-rate schedule");
}

// Workspace for steps of `batch` samples; allocates, so never called under capture.
static void reserve_step(Net& N, int32_t batch, int32_t n_steps, int g) {
  const int G = train_grid(batch, g);
  ensure_partials(N, G);
  N.xt.ensure(std::max<int64_t>(batch, 1));
  N.losses.ensure(std::max(n_steps, 1));
  N.ran.ensure(std::max(n_steps, 1));
}

// Enqueues optimiser step `step` (0-based within the phase) of every network in
// `groups` on `tree`: a gather per network, one fused train launch per group,
// one reduce + Adam launch for all.  Workspace must be reserved beforehand.
// `ev`, if non-null, holds two events per group around its train launch.
// The record of network k of model m for one training step on `tree` (n samples).
static void fill_train_net(nvdb_model* m, const Tree* tree, int k, const Phase& ph, int step, const StepHooks& hk,
                           TrainNet& tn) {
  Net& N = m->nets[k];
  tn.net = net_view(N);
  tn.tree = tree_view(tree);
  base_spec(m, &tn.spec);
  int64_t pop;
  tn.spec.src = population_src(k, tree, &pop);
  tn.spec.loss = (k == NVDB_NET_REGRESSOR || k == NVDB_NET_TILE) ? LOSS_MSE : (k == NVDB_NET_L0 ? LOSS_BCE : LOSS_CE);
  tn.spec.npop = (uint32_t)pop;
  int64_t n = ph.batch;
  if (ph.idx && ph.idx->idx_dev[k]) {
    const int64_t off = (int64_t)step * ph.batch;
    n = std::min<int64_t>(ph.batch, ph.idx->idx_count[k] - off);
    tn.spec.idx = ph.idx->idx_dev[k] + off;
    tn.spec.bad_idx = m->errw.p;
  } else {
    tn.spec.step_seed = step_seed(ph.seed, k, N.step);
  }
  tn.spec.n = n;
  tn.spec.inv_n = 1.f / (float)n;
  tn.prev_loss = hk.prev_loss[k];
  tn.stop_below = hk.stop_below[k];
  // the BF16 kernels draw i.i.d. samples over voxels or leaf slots themselves;
  // explicit index lists, the level-1 slots and the FP32 form use the gather kernel
  tn.fused = m->d.precision == NVDB_BF16 && !tn.spec.idx &&
             (tn.spec.src == SRC_VOXELS || tn.spec.src == SRC_LEAF_SLOTS);
  tn.partial = N.partial.p;
  tn.loss_partial = N.loss_partial.p;
  tn.xt = N.xt.p;
}

// The optimiser record of network k after a training launch of G work-groups.
static AdamNet fill_adam_net(nvdb_model* m, int k, const TrainNet& tn, int G, const Phase& ph, const StepHooks& hk) {
  Net& N = m->nets[k];
  NVDB_REQUIRE(N.partial.n >= (size_t)G * N.s.pstride() && N.xt.n >= (size_t)tn.spec.n, NVDB_E_STATE,
               "training workspace not reserved");
  const int64_t s = N.step + 1;
  AdamNet a = adam_view(N);
  a.partial = N.partial.p;
  a.loss_partial = N.loss_partial.p;
  a.G = G;
  a.loss_out = hk.loss_out[k];
  a.loss_scale = tn.spec.inv_n;
  a.lr = (float)((double)ph.lr * std::pow((double)ph.lr_decay, (double)((s - 1) / ph.lr_interval)));
  a.bc1 = (float)(1.0 - std::pow(0.9, (double)s));
  a.bc2 = (float)(1.0 - std::pow(0.999, (double)s));
  a.prev_loss = hk.prev_loss[k];
  a.stop_below = hk.stop_below[k];
  a.ran = hk.ran[k];
  a.grad_out = hk.grad_out[k];
  return a;
}

// One training step of the networks of `groups` (each group one launch of its kernel).
static void enqueue_step(nvdb_model* m, const Tree* tree, const std::vector<std::vector<int>>& groups,
                         const Phase& ph, int step, const StepHooks& hk, hipEvent_t* ev, hipStream_t st) {
  AdamLaunch AL{};
  int na = 0;
  int64_t maxP = 0;
  size_t evi = 0;
  for (auto& grp : groups) {
    NVDB_REQUIRE(grp.size() <= (size_t)MAX_LAUNCH_NETS, NVDB_E_INVALID, "too many networks for one launch");
    TrainLaunch L{};
    int G = 1;
    for (size_t i = 0; i < grp.size(); ++i) {
      fill_train_net(m, tree, grp[i], ph, step, hk, L.nets[i]);
      G = std::max(G, train_grid(L.nets[i].spec.n, m->train_g > 0 ? m->train_g : DEFAULT_G));
    }
    SampleSpec gspec[NVDB_MAX_NETS];
    floatx4* gout[NVDB_MAX_NETS];
    int ng = 0;
    for (size_t i = 0; i < grp.size(); ++i) {
      const int k = grp[i];
      if (!L.nets[i].fused) {
        gspec[ng] = L.nets[i].spec;
        gout[ng++] = m->nets[k].xt.p;
      }
      AL.nets[na++] = fill_adam_net(m, k, L.nets[i], G, ph, hk);
      maxP = std::max(maxP, m->nets[k].s.nparams());
    }
    L.G = G;
    if (ng > 0) launch_gather_multi(gspec, gout, ng, tree_view(tree), st);
    if (ev) NVDB_HIP(hipEventRecord(ev[evi++], st));
    launch_train(m->nets[grp[0]].ks, L, (int)grp.size(), st);
    if (ev) NVDB_HIP(hipEventRecord(ev[evi++], st));
  }
  launch_reduce_adam(AL, maxP, na, st);
  for (auto& grp : groups)
    for (int k : grp)
      if (!hk.grad_out[k]) m->nets[k].step += 1;
}

// One network of one model in a multi-model step.
struct StepUnit {
  nvdb_model* m;
  const Tree* tree;
  int k;
  int G;
};

// One training step of many models' networks (the experts of a decomposition):
// networks of one kernel and work-group count share launches of up to
// MAX_LAUNCH_NETS networks, each on its own tree; the optimiser launches take up
// to MAX_ADAM_NETS networks.  Per network the same arithmetic as enqueue_step.
static void enqueue_step_units(const std::vector<std::vector<StepUnit>>& launches, const Phase& ph, int step,
                               hipStream_t st) {
  std::vector<std::pair<AdamNet, int64_t>> adam;
  for (const auto& grp : launches) {
    TrainLaunch L{};
    const int G = grp[0].G;
    for (size_t i = 0; i < grp.size(); ++i) {
      const StepUnit& u = grp[i];
      StepHooks hk;
      hk.loss_out[u.k] = u.m->nets[u.k].losses.p + step;
      fill_train_net(u.m, u.tree, u.k, ph, step, hk, L.nets[i]);
      if (!L.nets[i].fused) {
        SampleSpec sp = L.nets[i].spec;
        floatx4* out = u.m->nets[u.k].xt.p;
        launch_gather_multi(&sp, &out, 1, tree_view(u.tree), st);
      }
      adam.push_back({fill_adam_net(u.m, u.k, L.nets[i], G, ph, hk), u.m->nets[u.k].s.nparams()});
    }
    L.G = G;
    launch_train(grp[0].m->nets[grp[0].k].ks, L, (int)grp.size(), st);
  }
  for (size_t a0 = 0; a0 < adam.size(); a0 += MAX_ADAM_NETS) {
    AdamLaunch AL{};
    int64_t maxP = 0;
    const size_t na = std::min<size_t>(MAX_ADAM_NETS, adam.size() - a0);
    for (size_t i = 0; i < na; ++i) {
      AL.nets[i] = adam[a0 + i].first;
      maxP = std::max(maxP, adam[a0 + i].second);
    }
    launch_reduce_adam(AL, maxP, (int)na, st);
  }
  for (const auto& grp : launches)
    for (const StepUnit& u : grp) u.m->nets[u.k].step += 1;
}

extern "C" {

nvdb_status nvdb_fit(nvdb_model* m, const nvdb_tree* tree, const nvdb_fit_desc* fit, float* loss_host, void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(m && tree && fit, NVDB_E_INVALID, "null argument");
    check_schedule(fit);
    hipStream_t st = (hipStream_t)stream;
    const std::vector<int> nets = fit_nets(m, tree, fit->nets_mask);
    for (int k : nets)
      if (fit->idx_dev[k])
        NVDB_REQUIRE(fit->idx_count[k] > (int64_t)(fit->steps - 1) * fit->batch, NVDB_E_INVALID,
                     "explicit index list shorter than the schedule");
    for (int k : nets) reserve_step(m->nets[k], fit->batch, fit->steps, m->train_g > 0 ? m->train_g : DEFAULT_G);
    const auto groups = kernel_groups(m, nets);
    const Phase ph{fit->batch, fit->seed, fit->lr, fit->lr_decay, fit->lr_interval, fit};

    // optional timing of the training-kernel launches with HIP events on `stream`
    const size_t n_ev = fit->train_kernel_ms ? 2 * (size_t)fit->steps * groups.size() : 0;
    if (n_ev) NVDB_HIP(hipStreamSynchronize(st));  // earlier timed fits may still use the cached events
    while (m->timing.size() < n_ev) {
      hipEvent_t e = nullptr;
      NVDB_HIP(hipEventCreate(&e));
      m->timing.push_back(e);
    }
    hipEvent_t* ev = n_ev ? m->timing.data() : nullptr;
    for (int step = 0; step < fit->steps; ++step) {
      StepHooks hk;
      for (int k : nets) hk.loss_out[k] = m->nets[k].losses.p + step;
      enqueue_step(m, tree, groups, ph, step, hk, ev ? ev + 2 * groups.size() * step : nullptr, st);
    }
    mark(m, st);
    bool lists = false;
    for (int k : nets) lists = lists || fit->idx_dev[k] != nullptr;
    if (lists) NVDB_REQUIRE(take_bad_indices(m) == 0, NVDB_E_INVALID, "sample index at or beyond its population size");
    if (n_ev) {
      NVDB_HIP(hipEventSynchronize(ev[n_ev - 1]));
      double tot = 0.0;
      for (size_t i = 0; i + 1 < n_ev; i += 2) {
        float ms = 0.f;
        NVDB_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
        tot += ms;
      }
      *fit->train_kernel_ms = (float)tot;
    }
    if (loss_host) {
      std::vector<float> h(std::max(fit->steps, 1));
      bool finite = true;
      for (int k : nets) {
        if (fit->steps == 0) break;
        NVDB_HIP(hipMemcpyAsync(h.data(), m->nets[k].losses.p, fit->steps * 4, hipMemcpyDeviceToHost, st));
        NVDB_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < fit->steps; ++i) {
          loss_host[k * fit->steps + i] = h[i];
          finite = finite && std::isfinite(h[i]);
        }
      }
      NVDB_REQUIRE(finite, NVDB_E_NUMERIC, "non-finite loss during fit");
    }
  });
}

nvdb_status nvdb_fit_experts(nvdb_model* const* models, const nvdb_tree* const* trees, int32_t n,
                             const nvdb_fit_desc* fit, float* loss_host, void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(models && trees && fit, NVDB_E_INVALID, "null argument");
    NVDB_REQUIRE(n >= 1 && n <= MOE_MAX_EXPERTS, NVDB_E_INVALID, "expert count outside [1, 4096]");
    for (int k = 0; k < NVDB_MAX_NETS; ++k)
      NVDB_REQUIRE(fit->idx_dev[k] == nullptr, NVDB_E_INVALID, "explicit sample orders are per model (nvdb_fit)");
    for (int e = 0; e < n; ++e) {
      NVDB_REQUIRE(models[e] && trees[e], NVDB_E_INVALID, "null expert or tree");
      for (int f = 0; f < e; ++f) NVDB_REQUIRE(models[f] != models[e], NVDB_E_INVALID, "a model listed twice");
    }
    check_schedule(fit);
    // every workspace first: a buffer grown while other experts' steps are queued
    // would free memory, and a free waits for the whole device
    std::vector<std::vector<int>> nets((size_t)n);
    for (int e = 0; e < n; ++e) {
      nets[e] = fit_nets(models[e], trees[e], fit->nets_mask);
      for (int k : nets[e])
        reserve_step(models[e]->nets[k], fit->batch, fit->steps,
                     models[e]->train_g > 0 ? models[e]->train_g : DEFAULT_G);
    }
    const Phase ph{fit->batch, fit->seed, fit->lr, fit->lr_decay, fit->lr_interval, nullptr};
    hipStream_t st = (hipStream_t)stream;
    // networks of one kernel and work-group count share launches (each on its own
    // tree), so a step of many small experts fills the GPU in one launch
    std::vector<std::vector<StepUnit>> launches;
    for (int e = 0; e < n; ++e)
      for (int k : nets[e]) {
        const StepUnit u{models[e], trees[e], k,
                         train_grid(fit->batch, models[e]->train_g > 0 ? models[e]->train_g : DEFAULT_G)};
        bool put = false;
        for (auto& grp : launches)
          if (grp.size() < (size_t)MAX_LAUNCH_NETS && grp[0].G == u.G &&
              grp[0].m->nets[grp[0].k].ks.train == u.m->nets[u.k].ks.train) {
            grp.push_back(u);
            put = true;
            break;
          }
        if (!put) launches.push_back({u});
      }
    for (int step = 0; step < fit->steps; ++step) enqueue_step_units(launches, ph, step, st);
    NVDB_HIP(hipStreamSynchronize(st));
    if (loss_host && fit->steps > 0) {
      std::vector<float> h((size_t)fit->steps);
      bool finite = true;
      for (int e = 0; e < n; ++e)
        for (int k : nets[e]) {
          NVDB_HIP(hipMemcpy(h.data(), models[e]->nets[k].losses.p, (size_t)fit->steps * 4, hipMemcpyDeviceToHost));
          for (int i = 0; i < fit->steps; ++i) {
            loss_host[((int64_t)e * NVDB_MAX_NETS + k) * fit->steps + i] = h[i];
            finite = finite && std::isfinite(h[i]);
          }
        }
      NVDB_REQUIRE(finite, NVDB_E_NUMERIC, "non-finite loss during an expert fit");
    }
  });
}

nvdb_status nvdb_autotune(nvdb_model* m, const nvdb_tree* tree, int32_t nets_mask, int32_t batch, int32_t reps,
                          nvdb_tune_report* report, void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(m && tree && batch >= 1 && batch <= (1 << 24) && reps >= 1 && reps <= 1000, NVDB_E_INVALID,
                 "bad autotune arguments");
    hipStream_t st = (hipStream_t)stream;
    const std::vector<int> nets = fit_nets(m, tree, nets_mask);
    const int tiles = (int)std::min<int64_t>(MAX_G, ((int64_t)batch + TRAIN_TILE - 1) / TRAIN_TILE);
    static const int cand_all[] = {32, 64, 128, 192, 256, 320, 384, 512};
    std::vector<int> gs;
    for (int g : cand_all)
      if (g <= tiles) gs.push_back(g);
    if (gs.empty() || gs.back() != tiles) gs.push_back(tiles);
    // training kernels: activations in registers, and activation rows where a network has them
    std::vector<int> kinds = {NVDB_TRAIN_REGISTERS};
    for (int k : nets)
      if (m->nets[k].ks.train_rows) {
        kinds.push_back(NVDB_TRAIN_ROWS);
        break;
      }
    std::vector<std::pair<int, int>> cands;  // (kernel, G)
    for (int kd : kinds)
      for (int g : gs) cands.push_back({kd, g});
    NVDB_REQUIRE((int)cands.size() <= NVDB_TUNE_MAX, NVDB_E_INVALID, "too many candidates");
    std::vector<DevBuf<float>> grads(NVDB_MAX_NETS);
    for (int k : nets) {
      reserve_step(m->nets[k], batch, 1, MAX_G);
      grads[k].alloc(m->nets[k].s.nparams());
    }
    const int saved_g = m->train_g;
    std::vector<void (*)(TrainLaunch)> saved_train(NVDB_MAX_NETS);
    std::vector<int64_t> saved_step(NVDB_MAX_NETS);
    for (int k : nets) {
      saved_step[k] = m->nets[k].step;
      saved_train[k] = m->nets[k].ks.train;
    }
    auto use_kind = [&](int kd) {
      for (int k : nets) {
        KernelSet& ks = m->nets[k].ks;
        ks.train = (kd == NVDB_TRAIN_ROWS && ks.train_rows) ? ks.train_rows : ks.train_classic;
      }
    };
    hipEvent_t e0, e1;
    NVDB_HIP(hipEventCreate(&e0));
    NVDB_HIP(hipEventCreate(&e1));
    size_t best = 0;
    float best_ms = 0.f;
    std::vector<float> times;
    try {
      const Phase ph{batch, 0x5eedull, 0.f, 1.f, 1, nullptr};
      StepHooks hk;
      for (int k : nets) hk.grad_out[k] = grads[k].p;
      for (size_t c = 0; c < cands.size(); ++c) {
        use_kind(cands[c].first);
        const auto groups = kernel_groups(m, nets);
        m->train_g = cands[c].second;
        enqueue_step(m, tree, groups, ph, 0, hk, nullptr, st);  // warm-up
        NVDB_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) enqueue_step(m, tree, groups, ph, 0, hk, nullptr, st);
        NVDB_HIP(hipEventRecord(e1, st));
        NVDB_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        NVDB_HIP(hipEventElapsedTime(&ms, e0, e1));
        ms /= (float)reps;
        times.push_back(ms);
        if (c == 0 || ms < best_ms) {
          best_ms = ms;
          best = c;
        }
      }
    } catch (...) {
      m->train_g = saved_g;
      for (int k : nets) m->nets[k].ks.train = saved_train[k];
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int k : nets) m->nets[k].step = saved_step[k];
    use_kind(cands[best].first);
    m->train_g = cands[best].second;
    if (report) {
      std::memset(report, 0, sizeof(*report));
      report->chosen_g = cands[best].second;
      report->chosen_kernel = cands[best].first;
      report->n_candidates = (int32_t)cands.size();
      for (size_t c = 0; c < cands.size(); ++c) {
        report->kernel[c] = cands[c].first;
        report->g[c] = cands[c].second;
        report->ms_per_step[c] = times[c];
      }
    }
  });
}

nvdb_status nvdb_model_set_train_kernel(nvdb_model* m, int32_t kind) {
  return guarded([&] {
    NVDB_REQUIRE(m && (kind == NVDB_TRAIN_REGISTERS || kind == NVDB_TRAIN_ROWS), NVDB_E_INVALID,
                 "unknown training kernel");
    wait_model(m);
    for (int k = 0; k < NVDB_MAX_NETS; ++k) {
      if (!m->nets[k].present) continue;
      KernelSet& ks = m->nets[k].ks;
      ks.train = (kind == NVDB_TRAIN_ROWS && ks.train_rows) ? ks.train_rows : ks.train_classic;
    }
  });
}

nvdb_status nvdb_model_set_train_groups(nvdb_model* m, int32_t g) {
  return guarded([&] {
    NVDB_REQUIRE(m && g >= 0 && g <= MAX_G, NVDB_E_INVALID, "work-groups per network must be in 0..512");
    m->train_g = g;
  });
}

}  // extern "C"

// Records a long run of launches as a series of HIP graphs of at most
// MAX_STEPS optimiser steps each, launched in order on the caller's stream.
// Graphs are kept to a few thousand nodes: the whole schedule of a long
// sequence (tens of thousands of steps, four launches each) recorded as one
// graph made the host runtime crash, while graphs of ~10^4 nodes ran.  Every
// executable graph stays alive until the caller has synchronised.
struct GraphChunks {
  static constexpr int MAX_STEPS = 512;
  hipStream_t main = nullptr, cs = nullptr;
  bool on = false, capturing = false;
  int steps = 0;
  std::vector<hipGraphExec_t> execs;
  GraphChunks(hipStream_t st, bool use) : main(st), on(use) {
    if (on) NVDB_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  }
  // stream on which the next operation is to be enqueued
  hipStream_t q() {
    if (!on) return main;
    if (!capturing) {
      NVDB_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      capturing = true;
    }
    return cs;
  }
  void step_done() {
    if (on && ++steps >= MAX_STEPS) flush();
  }
  void flush() {
    if (!capturing) return;
    capturing = false;
    steps = 0;
    hipGraph_t g = nullptr;
    NVDB_HIP(hipStreamEndCapture(cs, &g));
    hipGraphExec_t e = nullptr;
    const hipError_t r = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    NVDB_HIP(r);
    execs.push_back(e);
    NVDB_HIP(hipGraphLaunch(e, main));
  }
  ~GraphChunks() {
    if (capturing) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
    }
    if (!execs.empty()) (void)hipStreamSynchronize(main);
    for (auto e : execs) (void)hipGraphExecDestroy(e);
    if (cs) (void)hipStreamDestroy(cs);
  }
};

extern "C" {

nvdb_status nvdb_fit_sequence(nvdb_model* m, const nvdb_tree* const* frames, int32_t n_frames,
                              const nvdb_fit_desc* cold, const nvdb_fit_desc* warm, int32_t use_graph,
                              nvdb_frame_report* reports, float* loss_host, float* frame_params_dev,
                              void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(m && frames && cold && warm && n_frames >= 1, NVDB_E_INVALID, "null argument or no frames");
    check_schedule(cold);
    check_schedule(warm);
    NVDB_REQUIRE(cold->steps >= 1 && warm->steps >= 1, NVDB_E_INVALID, "cold and warm passes need >= 1 step");
    NVDB_REQUIRE(cold->nets_mask == warm->nets_mask, NVDB_E_INVALID, "cold and warm passes select other networks");
    for (int k = 0; k < NVDB_MAX_NETS; ++k)
      NVDB_REQUIRE(!cold->idx_dev[k] && !warm->idx_dev[k], NVDB_E_INVALID,
                   "sequences draw i.i.d. batches; explicit index lists are not accepted");
    std::vector<int> nets;
    for (int32_t f = 0; f < n_frames; ++f) {
      NVDB_REQUIRE(frames[f], NVDB_E_INVALID, "null frame");
      nets = fit_nets(m, frames[f], cold->nets_mask);
    }
    const int64_t total = (int64_t)cold->steps + (int64_t)n_frames * warm->steps;
    NVDB_REQUIRE(total < (1ll << 30), NVDB_E_INVALID, "schedule too long");
    for (int k : nets) {
      Net& N = m->nets[k];
      reserve_step(N, std::max(cold->batch, warm->batch), (int32_t)total, m->train_g > 0 ? m->train_g : DEFAULT_G);
    }
    const auto groups = kernel_groups(m, nets);
    hipStream_t st = (hipStream_t)stream;

    GraphChunks cap(st, use_graph != 0);
    int64_t frame_stride = 0;
    for (int k : nets) frame_stride += m->nets[k].s.nparams();
    int64_t g = 0;  // global step index into each network's loss / ran arrays
    // A pass starts from a fresh optimiser state: zero moments, step count 0.
    auto run_pass = [&](const Tree* tree, const nvdb_fit_desc* d, uint64_t seed, bool stop_test) {
      for (int k : nets) {
        Net& N = m->nets[k];
        launch_fill(N.m.p, N.s.nparams(), 0.f, cap.q());
        launch_fill(N.v.p, N.s.nparams(), 0.f, cap.q());
        N.step = 0;
      }
      const Phase ph{d->batch, seed, d->lr, d->lr_decay, d->lr_interval, nullptr};
      for (int j = 0; j < d->steps; ++j, ++g) {
        StepHooks hk;
        for (int k : nets) {
          Net& N = m->nets[k];
          hk.loss_out[k] = N.losses.p + g;
          hk.ran[k] = N.ran.p + g;
          if (stop_test && j > 0) {
            hk.prev_loss[k] = N.losses.p + g - 1;
            hk.stop_below[k] = N.losses.p + (cold->steps + warm->steps - 1);
          }
        }
        enqueue_step(m, tree, groups, ph, j, hk, nullptr, cap.q());
        cap.step_done();
      }
    };
    auto save_frame = [&](int32_t f) {
      if (!frame_params_dev) return;
      int64_t off = (int64_t)f * frame_stride;
      for (int k : nets) {
        Net& N = m->nets[k];
        NVDB_HIP(hipMemcpyAsync(frame_params_dev + off, N.theta.p, N.s.nparams() * 4, hipMemcpyDeviceToDevice,
                                cap.q()));
        off += N.s.nparams();
      }
    };
    // frame 0: cold pass at the target rate, then a refit at the warm rate (Sec. 3.6)
    run_pass(frames[0], cold, cold->seed, false);
    run_pass(frames[0], warm, warm->seed, false);
    save_frame(0);
    // later frames: warm start from the previous frame's weights, stopping once the
    // batch loss falls below frame 0's final loss
    for (int32_t f = 1; f < n_frames; ++f) {
      run_pass(frames[f], warm, warm->seed + (uint64_t)f, true);
      save_frame(f);
    }
    cap.flush();
    NVDB_HIP(hipStreamSynchronize(st));

    // per-frame report; the host step counters follow the steps that actually ran
    bool finite = true;
    std::vector<float> lh(total);
    std::vector<int32_t> rh(total);
    if (reports) std::memset(reports, 0, sizeof(nvdb_frame_report) * n_frames);
    for (int k : nets) {
      Net& N = m->nets[k];
      NVDB_HIP(hipMemcpy(lh.data(), N.losses.p, total * 4, hipMemcpyDeviceToHost));
      NVDB_HIP(hipMemcpy(rh.data(), N.ran.p, total * 4, hipMemcpyDeviceToHost));
      int64_t i = 0;
      int32_t last_run = 0;
      for (int32_t f = 0; f < n_frames; ++f) {
        const int64_t len = f == 0 ? (int64_t)cold->steps + warm->steps : warm->steps;
        int32_t run = 0;
        for (int64_t j = 0; j < len; ++j, ++i) {
          run += rh[i];
          finite = finite && std::isfinite(lh[i]);
        }
        if (reports) {
          reports[f].steps_run[k] = run;
          reports[f].final_loss[k] = lh[i - 1];
        }
        last_run = f == 0 ? run - cold->steps : run;
      }
      N.step = last_run;
      if (loss_host) std::memcpy(loss_host + (int64_t)k * total, lh.data(), total * 4);
    }
    NVDB_REQUIRE(finite, NVDB_E_NUMERIC, "non-finite loss during the sequence fit");
  });
}

// ------------------------------------------------------------------ decode
static int infer8_grid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 512)); }

}  // extern "C"

// Launches the forward pass of network N over one population of `tree`; the FP8
// form first requantises the weights from the master copy.
static void run_infer(const nvdb_model* m, const Net& N, const Tree* tree, int src, int64_t n, InferLaunch I, bool fp8,
                      hipStream_t st) {
  I.net = net_view(N);
  base_spec(m, &I.spec);
  I.spec.src = src;
  I.spec.direct = 1;
  I.spec.n = n;
  I.tree = tree_view(tree);
  if (fp8) {
    NVDB_REQUIRE(N.ks.infer8 != nullptr, NVDB_E_UNSUPPORTED, "no FP8 kernel for this network shape");
    N.w8.ensure((size_t)fp8_weight_bytes(N.s));
    N.w8inv.ensure(2 * (size_t)N.s.H);
    launch_quant_fp8(N.s, N.theta.p, N.w8.p, N.w8inv.p, st);
    I.w8 = N.w8.p;
    I.w8inv = N.w8inv.p;
    launch_infer8(N.ks, I, infer8_grid(n), st);
  } else {
    launch_infer(N.ks, I, infer_grid(N.ks, n), st);
  }
}

static void decode_impl(const nvdb_model* m, const nvdb_tree* tree, float* values_dev, uint64_t* pred_mask_dev,
                        bool fp8, hipStream_t st) {
  NVDB_REQUIRE(m && tree, NVDB_E_INVALID, "null argument");
  if (values_dev && tree->n_vox > 0) {
    const Net& N = net_of(m, NVDB_NET_REGRESSOR);
    NVDB_REQUIRE(N.params_set && N.enc_set, NVDB_E_STATE, "regressor parameters or encoding not set");
    InferLaunch I{};
    I.out_kind = OUT_VALUES;
    I.out_scale = m->d.value_scale;
    I.y = values_dev;
    run_infer(m, N, tree, SRC_VOXELS, tree->n_vox, I, fp8, st);
  }
  if (pred_mask_dev && tree->n_leaf > 0) {
    const Net& N = net_of(m, NVDB_NET_L0);
    NVDB_REQUIRE(N.params_set && N.enc_set, NVDB_E_STATE, "classifier parameters or encoding not set");
    InferLaunch I{};
    I.out_kind = OUT_MASK;
    I.mask = pred_mask_dev;
    run_infer(m, N, tree, SRC_LEAF_SLOTS, 512 * tree->n_leaf, I, fp8, st);
  }
}

extern "C" {

nvdb_status nvdb_autotune_decode(nvdb_model* m, const nvdb_tree* tree, int32_t nets_mask, int32_t reps,
                                 nvdb_decode_tune_report* report, void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(m && tree && reps >= 1 && reps <= 1000, NVDB_E_INVALID, "bad autotune arguments");
    hipStream_t st = (hipStream_t)stream;
    const std::vector<int> nets = fit_nets(m, tree, nets_mask);
    hipEvent_t e0, e1;
    NVDB_HIP(hipEventCreate(&e0));
    NVDB_HIP(hipEventCreate(&e1));
    if (report) std::memset(report, 0, sizeof(*report));
    int nc = 0;
    try {
      wait_model(m);
      for (int k : nets) {
        Net& N = m->nets[k];
        int64_t n;
        const int src = population_src(k, tree, &n);
        DevBuf<float> y;
        y.alloc(n * N.s.C);
        const int saved = N.ks.infer_sel;
        int best = 0;
        float best_ms = 0.f;
        for (int v = 0; v < N.ks.n_infer_v; ++v) {
          N.ks.infer_sel = v;
          InferLaunch I{};
          I.out_kind = OUT_Y;
          I.y = y.p;
          run_infer(m, N, tree, src, n, I, false, st);  // warm-up
          NVDB_HIP(hipEventRecord(e0, st));
          for (int r = 0; r < reps; ++r) run_infer(m, N, tree, src, n, I, false, st);
          NVDB_HIP(hipEventRecord(e1, st));
          NVDB_HIP(hipEventSynchronize(e1));
          float ms = 0.f;
          NVDB_HIP(hipEventElapsedTime(&ms, e0, e1));
          ms /= (float)reps;
          if (v == 0 || ms < best_ms) {
            best_ms = ms;
            best = v;
          }
          if (report && nc < NVDB_TUNE_MAX) {
            report->net[nc] = k;
            report->waves[nc] = N.ks.infer_v[v].waves;
            report->tiles[nc] = N.ks.infer_v[v].nt;
            report->ms[nc] = ms;
            ++nc;
          }
        }
        (void)saved;
        N.ks.infer_sel = best;
        if (report) report->chosen[k] = best;
      }
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (report) report->n_candidates = nc;
  });
}

nvdb_status nvdb_model_set_decode_shape(nvdb_model* m, int32_t net, int32_t index) {
  return guarded([&] {
    NVDB_REQUIRE(m, NVDB_E_INVALID, "null model");
    Net& N = net_of(m, net);
    NVDB_REQUIRE(index >= 0 && index < N.ks.n_infer_v, NVDB_E_INVALID, "no such decode tile shape");
    wait_model(m);
    N.ks.infer_sel = index;
  });
}

}  // extern "C"

static void decode_l1_impl(const nvdb_model* m, const nvdb_tree* tree, uint8_t* classes_dev, bool fp8, hipStream_t st) {
  NVDB_REQUIRE(m && tree && classes_dev, NVDB_E_INVALID, "null argument");
  const Net& N = net_of(m, NVDB_NET_L1);
  NVDB_REQUIRE(N.params_set && N.enc_set, NVDB_E_STATE, "level-1 classifier parameters or encoding not set");
  if (tree->n_l1 == 0) return;
  InferLaunch I{};
  I.out_kind = OUT_CLASS;
  I.cls = classes_dev;
  run_infer(m, N, tree, SRC_L1_SLOTS, 4096 * tree->n_l1, I, fp8, st);
}

// The tile value regressor at every active tile of `tree`, in value units.
static void decode_tiles_impl(const nvdb_model* m, const nvdb_tree* tree, float* values_dev, bool fp8,
                              hipStream_t st) {
  NVDB_REQUIRE(m && tree, NVDB_E_INVALID, "null argument");
  const Net& N = net_of(m, NVDB_NET_TILE);
  NVDB_REQUIRE(N.params_set && N.enc_set, NVDB_E_STATE, "tile value regressor parameters or encoding not set");
  if (tree->n_tile == 0) return;
  NVDB_REQUIRE(values_dev, NVDB_E_INVALID, "null argument");
  InferLaunch I{};
  I.out_kind = OUT_VALUES;
  I.out_scale = m->d.value_scale;
  I.y = values_dev;
  run_infer(m, N, tree, SRC_TILES, tree->n_tile, I, fp8, st);
}

extern "C" {

nvdb_status nvdb_decode_tiles(const nvdb_model* m, const nvdb_tree* tree, int32_t fp8, float* tile_values_dev,
                              void* stream) {
  return guarded([&] {
    decode_tiles_impl(m, tree, tile_values_dev, fp8 != 0, (hipStream_t)stream);
    mark(m, (hipStream_t)stream);
  });
}

nvdb_status nvdb_errors_tiles(const nvdb_tree* tree, const float* tile_values_dev, nvdb_error_report* out,
                              void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(tree && out && (tile_values_dev || tree->n_tile == 0), NVDB_E_INVALID, "null argument");
    error_report_tiles(*tree, tile_values_dev, out, (hipStream_t)stream);
  });
}

nvdb_status nvdb_decode(const nvdb_model* m, const nvdb_tree* tree, float* values_dev, uint64_t* pred_mask_dev,
                        void* stream) {
  return guarded([&] {
    decode_impl(m, tree, values_dev, pred_mask_dev, false, (hipStream_t)stream);
    mark(m, (hipStream_t)stream);
  });
}

nvdb_status nvdb_decode_fp8(const nvdb_model* m, const nvdb_tree* tree, float* values_dev, uint64_t* pred_mask_dev,
                            void* stream) {
  return guarded([&] {
    decode_impl(m, tree, values_dev, pred_mask_dev, true, (hipStream_t)stream);
    mark(m, (hipStream_t)stream);
  });
}

nvdb_status nvdb_decode_l1(const nvdb_model* m, const nvdb_tree* tree, uint8_t* classes_dev, void* stream) {
  return guarded([&] {
    decode_l1_impl(m, tree, classes_dev, false, (hipStream_t)stream);
    mark(m, (hipStream_t)stream);
  });
}

nvdb_status nvdb_decode_l1_fp8(const nvdb_model* m, const nvdb_tree* tree, uint8_t* classes_dev, void* stream) {
  return guarded([&] {
    decode_l1_impl(m, tree, classes_dev, true, (hipStream_t)stream);
    mark(m, (hipStream_t)stream);
  });
}

nvdb_status nvdb_errors(const nvdb_tree* tree, const float* values_dev, const uint64_t* pred_mask_dev,
                        nvdb_error_report* out, void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(tree && values_dev && out, NVDB_E_INVALID, "null argument");
    error_report(*tree, values_dev, pred_mask_dev, out, (hipStream_t)stream);
  });
}

}  // extern "C"

// The lower tree levels decoded below the level-1 nodes of `upper` (see
// nvdb_decode_topology); synchronises `st`.
// leaf_masks (device, n_leaf_given x 8 words, canonical leaf order) replaces the
// level-0 inference when the leaf masks are stored explicitly.
static nvdb_tree* decode_topology_impl(const nvdb_model* m, const nvdb_tree* upper, bool use_fp8, hipStream_t st,
                                       const uint64_t* leaf_masks = nullptr, int64_t n_leaf_given = 0) {
  {
    const Net& R = net_of(m, NVDB_NET_REGRESSOR);
    NVDB_REQUIRE(R.params_set && R.enc_set, NVDB_E_STATE, "regressor parameters or encoding not set");
    const bool masks_given = leaf_masks != nullptr;
    const bool has_l0 = !masks_given && m->nets[NVDB_NET_L0].present;
    if (has_l0)
      NVDB_REQUIRE(m->nets[NVDB_NET_L0].params_set && m->nets[NVDB_NET_L0].enc_set, NVDB_E_STATE,
                   "level-0 classifier parameters or encoding not set");
    nvdb_tree* t = new nvdb_tree();
    try {
      for (int d = 0; d < 3; ++d) {
        t->origin[d] = upper->origin[d];
        t->dims[d] = upper->dims[d];
      }
      t->kind = upper->kind;
      t->thr = upper->thr;
      t->n_l1 = upper->n_l1;
      t->n_l2 = upper->n_l2;
      t->l2_origin = upper->l2_origin;
      const int64_t nl1 = std::max<int64_t>(t->n_l1, 1);
      t->l1_o.alloc(nl1);
      t->l1_child.alloc(nl1 * 64);
      t->l1_active.alloc(nl1 * 64);
      if (t->n_l1 > 0)
        NVDB_HIP(hipMemcpyAsync(t->l1_o.p, upper->l1_o.p, t->n_l1 * sizeof(int4), hipMemcpyDeviceToDevice, st));
      // level 1: classes of every leaf slot, predicted leaves
      const int64_t n_slots = 4096 * t->n_l1;
      DevBuf<uint8_t> cls;
      DevBuf<uint64_t> flag, prefix;
      cls.alloc(std::max<int64_t>(n_slots, 1));
      flag.alloc(std::max<int64_t>(n_slots, 1));
      prefix.alloc(std::max<int64_t>(n_slots, 1));
      if (n_slots > 0) {
        // level-1 classes from the level-1 classifier, or, for a model without one,
        // from the child and tile masks `upper` stores explicitly
        if (m->nets[NVDB_NET_L1].present) decode_l1_impl(m, upper, cls.p, use_fp8, st);
        else classes_from_masks(*upper, cls.p, st);
        pred_flags(cls.p, n_slots, flag.p, st);
      }
      const uint64_t nleaf = scan_u64(flag.p, n_slots, prefix.p, st);
      t->n_leaf = (int64_t)nleaf;
      t->leaf_o.alloc(std::max<int64_t>(t->n_leaf, 1));
      t->leaf_mask.alloc(std::max<int64_t>(t->n_leaf, 1) * 8);
      t->leaf_off.alloc(t->n_leaf + 1);
      if (n_slots > 0) pred_leaves(cls.p, prefix.p, t->l1_o.p, n_slots, t->leaf_o.p, t->l1_child.p, t->l1_active.p, st);
      // active tiles: the slots of the active-tile class, valued by the tile regressor
      const Net& TR = m->nets[NVDB_NET_TILE];
      if (TR.present) {
        NVDB_REQUIRE(TR.params_set && TR.enc_set, NVDB_E_STATE, "tile value regressor parameters or encoding not set");
        tiles_from_classes(cls.p, n_slots, t, st);
        decode_tiles_impl(m, t, t->tile_val.p, use_fp8, st);
      }
      // level 0: voxel masks
      DevBuf<float> slot_y;
      if (masks_given) {
        NVDB_REQUIRE(t->n_leaf == n_leaf_given, NVDB_E_INVALID, "stored leaf masks do not match the level-1 masks");
        if (t->n_leaf > 0)
          NVDB_HIP(hipMemcpyAsync(t->leaf_mask.p, leaf_masks, t->n_leaf * 64, hipMemcpyDeviceToDevice, st));
      } else if (t->n_leaf > 0) {
        if (has_l0) {
          InferLaunch I{};
          I.out_kind = OUT_MASK;
          I.mask = t->leaf_mask.p;
          run_infer(m, m->nets[NVDB_NET_L0], t, SRC_LEAF_SLOTS, 512 * t->n_leaf, I, use_fp8, st);
        } else {
          slot_y.alloc(512 * t->n_leaf);
          InferLaunch I{};
          I.out_kind = OUT_Y;
          I.y = slot_y.p;
          run_infer(m, R, t, SRC_LEAF_SLOTS, 512 * t->n_leaf, I, use_fp8, st);
          mask_from_values(slot_y.p, t->n_leaf, m->d.value_scale, t->kind, t->thr, t->leaf_mask.p, st);
        }
      }
      const bool values_from_slots = !has_l0 && !masks_given;
      pred_voxels(t->leaf_mask.p, t->n_leaf, t, values_from_slots ? slot_y.p : nullptr, m->d.value_scale, st);
      // values at the predicted voxels
      if (!values_from_slots && t->n_vox > 0) {
        InferLaunch I{};
        I.out_kind = OUT_VALUES;
        I.out_scale = m->d.value_scale;
        I.y = t->values.p;
        run_infer(m, R, t, SRC_VOXELS, t->n_vox, I, use_fp8, st);
      }
      NVDB_HIP(hipStreamSynchronize(st));
    } catch (...) {
      delete t;
      throw;
    }
    return t;
  }
}

extern "C" {

nvdb_status nvdb_decode_topology(const nvdb_model* m, const nvdb_tree* upper, int32_t fp8, nvdb_tree** out,
                                 void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(m && upper && out, NVDB_E_INVALID, "null argument");
    *out = nullptr;
    *out = decode_topology_impl(m, upper, fp8 != 0, (hipStream_t)stream);
  });
}

nvdb_status nvdb_errors_topology(const nvdb_tree* truth, const nvdb_tree* pred, nvdb_topology_report* out,
                                 void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(truth && pred && out, NVDB_E_INVALID, "null argument");
    NVDB_REQUIRE(truth->n_l1 == pred->n_l1, NVDB_E_INVALID, "trees do not share their level-1 nodes");
    error_report_topology(*truth, *pred, out, (hipStream_t)stream);
  });
}

nvdb_status nvdb_errors_l1(const nvdb_tree* tree, const uint8_t* classes_dev, nvdb_l1_report* out, void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(tree && out && (classes_dev || tree->n_l1 == 0), NVDB_E_INVALID, "null argument");
    error_report_l1(*tree, classes_dev, out, (hipStream_t)stream);
  });
}

// ------------------------------------------------------------------ device-pointer calls
nvdb_status nvdb_query(const nvdb_model* m, const nvdb_tree* tree, const float* q_dev, int64_t n, float background,
                       int64_t batch, float* values_dev, uint8_t* hits_dev, void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(m && tree, NVDB_E_INVALID, "null argument");
    NVDB_REQUIRE(n >= 0 && (n == 0 || (q_dev && values_dev)), NVDB_E_INVALID, "bad buffers");
    NVDB_REQUIRE(batch >= 0 && n < (1ll << 31), NVDB_E_INVALID, "bad query count or batch");
    NVDB_REQUIRE(std::isfinite(background), NVDB_E_INVALID, "background must be finite");
    const Net& N = net_of(m, NVDB_NET_REGRESSOR);
    NVDB_REQUIRE(N.params_set && N.enc_set, NVDB_E_STATE, "regressor parameters or encoding not set");
    // active tiles are looked up when the tree has them and the model holds the tile regressor
    const Net& TN = m->nets[NVDB_NET_TILE];
    const bool tiles = tree->n_tile > 0 && TN.present;
    if (tiles) NVDB_REQUIRE(TN.params_set && TN.enc_set, NVDB_E_STATE, "tile value regressor parameters or encoding not set");
    if (n == 0) return;
    hipStream_t st = (hipStream_t)stream;
    const int64_t bs = batch > 0 ? std::min<int64_t>(batch, n) : n;
    DevBuf<float> hit_x, y, tile_x, tile_y;
    DevBuf<uint32_t> hit_idx, cnt, tile_idx;
    hit_x.alloc(3 * (size_t)bs);
    y.alloc((size_t)bs);
    hit_idx.alloc((size_t)bs);
    cnt.alloc(2);
    QueryTiles qt{};
    if (tiles) {
      tile_x.alloc(3 * (size_t)bs);
      tile_y.alloc((size_t)bs);
      tile_idx.alloc((size_t)bs);
      qt = QueryTiles{tree->l1_o.p, tree->l1_active.p, tree->n_l1, tile_x.p, tile_idx.p, cnt.p + 1};
    }
    const float inv_d = 1.f / (float)m->d.domain_size;
    for (int64_t b0 = 0; b0 < n; b0 += bs) {
      const int64_t nb = std::min(bs, n - b0);
      query_zero_count(cnt.p, st);
      if (tiles) query_zero_count(cnt.p + 1, st);
      query_classify(q_dev + 3 * b0, nb, *tree, background, m->d.domain_lo, inv_d, values_dev + b0,
                     hits_dev ? hits_dev + b0 : nullptr, hit_x.p, hit_idx.p, cnt.p, qt, st);
      if (tiles) {  // the tile regressor over the batch's tile hits (count read on the device)
        InferLaunch T{};
        T.net = net_view(TN);
        base_spec(m, &T.spec);
        T.spec.src = SRC_COORDS;
        T.spec.direct = 1;
        T.spec.coords = tile_x.p;
        T.spec.n = nb;
        T.spec.n_dev = cnt.p + 1;
        T.out_kind = OUT_Y;
        T.y = tile_y.p;
        launch_infer(TN.ks, T, infer_grid(TN.ks, nb), st);
        query_scatter(tile_y.p, tile_idx.p, nb, cnt.p + 1, m->d.value_scale, values_dev + b0, st);
      }
      // the regressor over the batch's hits: launched for nb samples, it reads the
      // hit count on the device (waves past it exit at once)
      InferLaunch I{};
      I.net = net_view(N);
      base_spec(m, &I.spec);
      I.spec.src = SRC_COORDS;
      I.spec.direct = 1;
      I.spec.coords = hit_x.p;
      I.spec.n = nb;
      I.spec.n_dev = cnt.p;
      I.out_kind = OUT_Y;
      I.y = y.p;
      launch_infer(N.ks, I, infer_grid(N.ks, nb), st);
      query_scatter(y.p, hit_idx.p, nb, cnt.p, m->d.value_scale, values_dev + b0, st);
    }
    NVDB_HIP(hipStreamSynchronize(st));
  });
}

nvdb_status nvdb_query_noalloc(const nvdb_model* m, const nvdb_tree* tree, const float* q_dev, int64_t n,
                               float background, int64_t batch, float* values_dev, uint8_t* hits_dev, void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(m && tree, NVDB_E_INVALID, "null argument");
    NVDB_REQUIRE(n >= 0 && (n == 0 || (q_dev && values_dev)), NVDB_E_INVALID, "bad buffers");
    NVDB_REQUIRE(n < (1ll << 31), NVDB_E_INVALID, "bad query count");
    NVDB_REQUIRE(batch >= 0 && batch <= QUERY_NOALLOC_MAX_BATCH, NVDB_E_INVALID,
                 "batch must be in 0..65536 (the static scratch holds one batch)");
    NVDB_REQUIRE(std::isfinite(background), NVDB_E_INVALID, "background must be finite");
    const Net& N = net_of(m, NVDB_NET_REGRESSOR);
    NVDB_REQUIRE(N.params_set && N.enc_set, NVDB_E_STATE, "regressor parameters or encoding not set");
    const Net& TN = m->nets[NVDB_NET_TILE];
    const bool tiles = tree->n_tile > 0 && TN.present;
    if (tiles) NVDB_REQUIRE(TN.params_set && TN.enc_set, NVDB_E_STATE, "tile value regressor parameters or encoding not set");
    if (n == 0) return;
    hipStream_t st = (hipStream_t)stream;
    const QueryScratch qs = query_noalloc_scratch();
    const int64_t bs = std::min<int64_t>(batch > 0 ? batch : QUERY_NOALLOC_MAX_BATCH, n);
    const float inv_d = 1.f / (float)m->d.domain_size;
    const QueryTiles qt =
        tiles ? QueryTiles{tree->l1_o.p, tree->l1_active.p, tree->n_l1, qs.tile_x, qs.tile_idx, qs.cnt + 1} : QueryTiles{};
    // batches run one after the other on `stream` and reuse the same scratch
    for (int64_t b0 = 0; b0 < n; b0 += bs) {
      const int64_t nb = std::min(bs, n - b0);
      query_zero_count(qs.cnt, st);
      if (tiles) query_zero_count(qs.cnt + 1, st);
      query_classify(q_dev + 3 * b0, nb, *tree, background, m->d.domain_lo, inv_d, values_dev + b0,
                     hits_dev ? hits_dev + b0 : nullptr, qs.hit_x, qs.hit_idx, qs.cnt, qt, st);
      if (tiles) {  // as in nvdb_query: the tile regressor over the batch's tile hits
        InferLaunch T{};
        T.net = net_view(TN);
        base_spec(m, &T.spec);
        T.spec.src = SRC_COORDS;
        T.spec.direct = 1;
        T.spec.coords = qs.tile_x;
        T.spec.n = nb;
        T.spec.n_dev = qs.cnt + 1;
        T.out_kind = OUT_Y;
        T.y = qs.tile_y;
        launch_infer(TN.ks, T, infer_grid(TN.ks, nb), st);
        query_scatter(qs.tile_y, qs.tile_idx, nb, qs.cnt + 1, m->d.value_scale, values_dev + b0, st);
      }
      InferLaunch I{};
      I.net = net_view(N);
      base_spec(m, &I.spec);
      I.spec.src = SRC_COORDS;
      I.spec.direct = 1;
      I.spec.coords = qs.hit_x;
      I.spec.n = nb;
      I.spec.n_dev = qs.cnt;
      I.out_kind = OUT_Y;
      I.y = qs.y;
      launch_infer(N.ks, I, infer_grid(N.ks, nb), st);
      query_scatter(qs.y, qs.hit_idx, nb, qs.cnt, m->d.value_scale, values_dev + b0, st);
    }
    mark(m, st);
  });
}

nvdb_status nvdb_topology_patches(const nvdb_tree* truth, const nvdb_tree* pred, int32_t* fp_dev, int64_t fp_cap,
                                  int32_t* fn_dev, int64_t fn_cap, int64_t* n_fp, int64_t* n_fn, void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(truth && pred && n_fp && n_fn, NVDB_E_INVALID, "null argument");
    NVDB_REQUIRE(fp_cap >= 0 && fn_cap >= 0 && (fp_cap == 0 || fp_dev) && (fn_cap == 0 || fn_dev), NVDB_E_INVALID,
                 "bad patch buffers");
    hipStream_t st = (hipStream_t)stream;
    *n_fp = topology_patches(*pred, *truth, fp_dev, fp_cap, st);
    *n_fn = topology_patches(*truth, *pred, fn_dev, fn_cap, st);
  });
}

// -------------------------------------------- sparse domain decomposition
}  // extern "C"

static MoeGrid check_grid(const nvdb_subdomains* g) {
  NVDB_REQUIRE(g != nullptr, NVDB_E_INVALID, "null subdomain grid");
  NVDB_REQUIRE(g->halo >= 1 && g->size >= 2 * g->halo && g->size <= (1 << 24), NVDB_E_INVALID,
               "subdomains need 1 <= halo and 2 halo <= size <= 2^24");
  MoeGrid m{};
  for (int d = 0; d < 3; ++d) {
    NVDB_REQUIRE(g->origin[d] >= -(1 << 24) && g->origin[d] <= (1 << 24), NVDB_E_INVALID,
                 "subdomain origin outside [-2^24, 2^24]");
    m.o[d] = g->origin[d];
  }
  m.S = g->size;
  m.h = g->halo;
  return m;
}
// Scratch of the blended decode, one per device, grown on demand and kept until
// the process ends (never freed: the runtime may be gone at exit).  A call holds
// its device's lock from the first use to its final synchronisation.
struct MoeScratch {
  std::mutex mu;
  DevBuf<uint8_t> small, big;
  // pinned host staging of the small arrays (uploaded with one asynchronous copy)
  uint8_t* host = nullptr;
  size_t host_cap = 0;
  uint8_t* host_buf(size_t n) {
    if (n > host_cap) {
      if (host) NVDB_HIP(hipHostFree(host));
      host = nullptr;
      host_cap = 0;
      NVDB_HIP(hipHostMalloc((void**)&host, n, hipHostMallocDefault));
      host_cap = n;
    }
    return host;
  }
};
static MoeScratch& moe_scratch() {
  static std::mutex m;
  static std::map<int, MoeScratch*> per_device;
  int dev = 0;
  NVDB_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(m);
  MoeScratch*& s = per_device[dev];
  if (!s) s = new MoeScratch();
  return *s;
}
// Waits for the stream when a call leaves early, so that its kernels are done
// with the shared scratch before the lock is released.
struct StreamDrain {
  hipStream_t st;
  ~StreamDrain() { (void)hipStreamSynchronize(st); }
};

static int64_t floor_div64(int64_t a, int64_t s) { return a >= 0 ? a / s : -((-a + s - 1) / s); }
static int64_t cell_range_size(const MoeGrid& g) { return (int64_t)g.cdim[0] * g.cdim[1] * g.cdim[2]; }
static constexpr int64_t MOE_MAX_RANGE = 1ll << 24;

extern "C" {

nvdb_status nvdb_subdomain_cells(const nvdb_tree* tree, const nvdb_subdomains* grid, int32_t* cells, int64_t cap,
                                 int64_t* n_cells, void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(tree && n_cells, NVDB_E_INVALID, "null argument");
    NVDB_REQUIRE(cap >= 0 && (cap == 0 || cells), NVDB_E_INVALID, "bad cell buffer");
    MoeGrid g = check_grid(grid);
    *n_cells = 0;
    if (tree->n_vox == 0 && tree->n_tile == 0) return;
    hipStream_t st = (hipStream_t)stream;
    int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    if (tree->n_leaf > 0) leaf_bbox(*tree, lo, hi, st);
    if (tree->n_tile > 0) {  // the active tiles lie in the level-1 nodes
      std::vector<int4> l1((size_t)tree->n_l1);
      NVDB_HIP(hipMemcpyAsync(l1.data(), tree->l1_o.p, l1.size() * sizeof(int4), hipMemcpyDeviceToHost, st));
      NVDB_HIP(hipStreamSynchronize(st));
      for (const int4& o : l1) {
        const int32_t c[3] = {o.x, o.y, o.z};
        for (int d = 0; d < 3; ++d) {
          lo[d] = std::min(lo[d], c[d]);
          hi[d] = std::max(hi[d], c[d] + 128);
        }
      }
    }
    for (int d = 0; d < 3; ++d) {
      const int64_t a = floor_div64((int64_t)lo[d] - g.o[d], g.S), b = floor_div64((int64_t)hi[d] - 1 - g.o[d], g.S);
      NVDB_REQUIRE(b - a + 1 <= MOE_MAX_RANGE, NVDB_E_INVALID, "the tree spans more than 2^24 cells");
      g.clo[d] = (int32_t)a;
      g.cdim[d] = (int32_t)(b - a + 1);
    }
    const int64_t total = cell_range_size(g);
    NVDB_REQUIRE(total <= MOE_MAX_RANGE, NVDB_E_INVALID, "the tree spans more than 2^24 cells");
    DevBuf<uint8_t> flag;
    flag.alloc((size_t)total);
    NVDB_HIP(hipMemsetAsync(flag.p, 0, (size_t)total, st));
    moe_mark_cells(*tree, g, flag.p, st);
    std::vector<uint8_t> h((size_t)total);
    NVDB_HIP(hipMemcpyAsync(h.data(), flag.p, (size_t)total, hipMemcpyDeviceToHost, st));
    NVDB_HIP(hipStreamSynchronize(st));
    int64_t c = 0;
    for (int64_t i = 0; i < total; ++i) {
      if (!h[i]) continue;
      if (c < cap) {
        cells[3 * c] = g.clo[0] + (int32_t)(i / ((int64_t)g.cdim[1] * g.cdim[2]));
        cells[3 * c + 1] = g.clo[1] + (int32_t)((i / g.cdim[2]) % g.cdim[1]);
        cells[3 * c + 2] = g.clo[2] + (int32_t)(i % g.cdim[2]);
      }
      ++c;
    }
    *n_cells = c;
  });
}

}  // extern "C"

// Lower corner of the widened box of `cell` (its expert's normalisation box).
static void widened_lo(const MoeGrid& g, const int32_t cell[3], int32_t lo[3]) {
  for (int d = 0; d < 3; ++d) {
    const int64_t l = (int64_t)g.o[d] + (int64_t)cell[d] * g.S - g.h;
    NVDB_REQUIRE(l >= -(1ll << 30) && l <= (1ll << 30), NVDB_E_INVALID, "cell outside the index range");
    lo[d] = (int32_t)l;
  }
}

extern "C" {

nvdb_status nvdb_subdomain_box(const nvdb_subdomains* grid, const int32_t cell[3], int32_t lo[3], int32_t* size) {
  return guarded([&] {
    NVDB_REQUIRE(cell && lo && size, NVDB_E_INVALID, "null argument");
    const MoeGrid g = check_grid(grid);
    widened_lo(g, cell, lo);
    *size = g.S + 2 * g.h;
  });
}

nvdb_status nvdb_tree_subdomain(const nvdb_tree* tree, const nvdb_subdomains* grid, const int32_t cell[3],
                                void* stream, nvdb_tree** out) {
  return guarded([&] {
    NVDB_REQUIRE(tree && cell && out, NVDB_E_INVALID, "null argument");
    *out = nullptr;
    const MoeGrid g = check_grid(grid);
    int32_t lo[3];
    widened_lo(g, cell, lo);
    hipStream_t st = (hipStream_t)stream;
    DevBuf<int32_t> ijk;
    DevBuf<float> v;
    DevBuf<uint32_t> count;
    const int64_t cap = std::max<int64_t>(tree->n_vox + 512 * tree->n_tile, 1);
    ijk.alloc(3 * (size_t)cap);
    v.alloc((size_t)cap);
    count.alloc(1);
    const int64_t n = moe_extract(*tree, lo, g.S + 2 * g.h, ijk.p, v.p, count.p, st);
    // every voxel of the source is kept: a band no finite value exceeds
    const nvdb_active_rule keep{NVDB_SDF, FLT_MAX};
    std::unique_ptr<Tree> t(build_tree_sparse(ijk.p, v.p, n, keep, st));
    t->kind = tree->kind;
    t->thr = tree->thr;
    // a source with active tiles: the tiles wholly inside the box become tiles again
    // (the source's leaves are never full and of one value, so no other leaf is pruned)
    if (tree->n_tile > 0) t.reset(prune_tiles(*t, st));
    *out = static_cast<nvdb_tree*>(t.release());
  });
}

}  // extern "C"

// Blended decode over the active voxels (regressors, values), over every voxel
// slot of the leaves (level-0 classifiers, mask bits), over every leaf slot of
// the level-1 nodes (level-1 classifiers, classes) or over the active tiles (tile
// value regressors, values).
static void decode_moe_impl(const nvdb_model* const* experts, const int32_t* cells, int32_t n_experts,
                            const nvdb_subdomains* grid, const nvdb_tree* tree, int net, float* values_dev,
                            uint64_t* mask_dev, uint8_t* cls_dev, hipStream_t st) {
  NVDB_REQUIRE(experts && cells && tree, NVDB_E_INVALID, "null argument");
  NVDB_REQUIRE(n_experts >= 1 && n_experts <= MOE_MAX_EXPERTS, NVDB_E_INVALID, "expert count outside [1, 4096]");
  const bool slots = net == NVDB_NET_L0;
  const int kind = net == NVDB_NET_REGRESSOR ? MOE_VOXELS
                   : net == NVDB_NET_L0      ? MOE_VOXEL_SLOTS
                   : net == NVDB_NET_L1      ? MOE_LEAF_SLOTS
                                             : MOE_TILES;
  const bool valued = kind == MOE_VOXELS || kind == MOE_TILES;  // value outputs, in value units
  const int64_t n = kind == MOE_VOXELS        ? tree->n_vox
                    : kind == MOE_VOXEL_SLOTS ? 512 * tree->n_leaf
                    : kind == MOE_LEAF_SLOTS  ? 4096 * tree->n_l1
                                              : tree->n_tile;
  const int C = kind == MOE_LEAF_SLOTS ? 3 : 1;
  NVDB_REQUIRE(n < (1ll << 29), NVDB_E_INVALID, "the blended decode takes fewer than 2^29 voxels or slots");
  NVDB_REQUIRE(n == 0 || (valued ? values_dev != nullptr
                                 : (kind == MOE_VOXEL_SLOTS ? mask_dev != nullptr : cls_dev != nullptr)),
               NVDB_E_INVALID, "null output");
  MoeGrid g = check_grid(grid);
  if (kind != MOE_VOXELS)
    NVDB_REQUIRE(g.S % 8 == 0 && g.o[0] % 8 == 0 && g.o[1] % 8 == 0 && g.o[2] % 8 == 0, NVDB_E_INVALID,
                 "the slot decodes need a cell size and grid origin that are multiples of 8");
  if (kind == MOE_LEAF_SLOTS || kind == MOE_TILES)
    NVDB_REQUIRE(g.h % 8 == 0, NVDB_E_INVALID, "the level-1 and tile decodes need a halo that is a multiple of 8");
  std::vector<MoeBox> box((size_t)n_experts);
  for (int k = 0; k < n_experts; ++k) {
    NVDB_REQUIRE(experts[k] != nullptr, NVDB_E_INVALID, "null expert");
    const Net& N = net_of(experts[k], net);
    NVDB_REQUIRE(N.params_set && N.enc_set, NVDB_E_STATE, "expert network parameters or encoding not set");
    NVDB_REQUIRE(N.s.C == C, NVDB_E_INVALID, "expert output count");
    for (int d = 0; d < 3; ++d) box[k].lo[d] = experts[k]->d.domain_lo[d];
    box[k].inv_d = 1.f / (float)experts[k]->d.domain_size;
  }
  int64_t clo[3], chi[3];
  for (int d = 0; d < 3; ++d) {
    clo[d] = chi[d] = cells[d];
    for (int k = 1; k < n_experts; ++k) {
      clo[d] = std::min<int64_t>(clo[d], cells[3 * k + d]);
      chi[d] = std::max<int64_t>(chi[d], cells[3 * k + d]);
    }
    NVDB_REQUIRE(chi[d] - clo[d] + 1 <= MOE_MAX_RANGE, NVDB_E_INVALID, "experts span more than 2^24 cells");
    g.clo[d] = (int32_t)clo[d];
    g.cdim[d] = (int32_t)(chi[d] - clo[d] + 1);
  }
  const int64_t total = cell_range_size(g);
  NVDB_REQUIRE(total <= MOE_MAX_RANGE, NVDB_E_INVALID, "experts span more than 2^24 cells");
  std::vector<int32_t> table((size_t)total, -1);
  for (int k = 0; k < n_experts; ++k) {
    const int64_t i =
        ((cells[3 * k] - clo[0]) * (int64_t)g.cdim[1] + (cells[3 * k + 1] - clo[1])) * g.cdim[2] + (cells[3 * k + 2] - clo[2]);
    NVDB_REQUIRE(table[(size_t)i] < 0, NVDB_E_INVALID, "two experts for one cell");
    table[(size_t)i] = k;
  }
  if (n == 0) return;
  const size_t E = (size_t)n_experts;
  // experts of one network shape decode in one grouped launch; the counts stay on
  // the device (no host round trip), the pair buffers are sized for the most pairs
  // possible (8 per item, each expert's run padded to whole chunks)
  const KernelSet& ks0 = net_of(experts[0], net).ks;
  bool grouped = ks0.infer_group != nullptr;
  for (size_t k = 1; k < E && grouped; ++k) grouped = net_of(experts[k], net).ks.infer_group == ks0.infer_group;
  if (grouped) {
    const size_t CH = (size_t)ks0.group_chunk;
    const size_t o_box = ((size_t)total * 4 + 255) & ~(size_t)255;
    const size_t o_cnt = o_box + ((E * sizeof(MoeBox) + 255) & ~(size_t)255);
    const size_t o_cs = o_cnt + (((E + 1) * 4 + 255) & ~(size_t)255);
    const size_t o_start = o_cs + (((E + 1) * 4 + 255) & ~(size_t)255);
    const size_t o_cur = o_start + ((E * 4 + 255) & ~(size_t)255);
    const size_t o_flag = o_cur + ((E * 4 + 255) & ~(size_t)255);
    const size_t o_nets = o_flag + 256;
    MoeScratch& ws = moe_scratch();
    std::lock_guard<std::mutex> lock(ws.mu);
    StreamDrain drain{st};  // declared after the lock: runs before it is released
    const size_t small_bytes = o_nets + E * sizeof(GroupNet);
    ws.small.ensure(small_bytes);
    uint8_t* small = ws.small.p;
    int32_t* tab = (int32_t*)small;
    MoeBox* dbox = (MoeBox*)(small + o_box);
    uint32_t* cnt = (uint32_t*)(small + o_cnt);
    uint32_t* cs = (uint32_t*)(small + o_cs);
    uint32_t* start = (uint32_t*)(small + o_start);
    uint32_t* cursor = (uint32_t*)(small + o_cur);
    uint32_t* flag = (uint32_t*)(small + o_flag);
    GroupNet* gnets = (GroupNet*)(small + o_nets);
    // the small arrays staged in pinned memory in their device layout, one upload
    uint8_t* hs = ws.host_buf(small_bytes + 256);
    std::memcpy(hs, table.data(), (size_t)total * 4);
    std::memcpy(hs + o_box, box.data(), E * sizeof(MoeBox));
    for (size_t k = 0; k < E; ++k) {
      GroupNet gn{};
      gn.net = net_view(net_of(experts[k], net));
      gn.out_scale = valued ? experts[k]->d.value_scale : 1.f;
      std::memcpy(hs + o_nets + k * sizeof(GroupNet), &gn, sizeof(GroupNet));
    }
    // the counters and cursors start at zero: the upload clears them
    std::memset(hs + o_cnt, 0, (E + 1) * 4);
    std::memset(hs + o_cur, 0, E * 4);
    uint32_t* back = (uint32_t*)(hs + small_bytes);  // overflow flag, uncovered items
    // pair buffers for two pairs per item (plus each run's padding to whole
    // chunks); if the routing finds more, the exact size is read back and the
    // decode runs again
    size_t cap = 2 * (size_t)n + E * CH;
    NVDB_REQUIRE(net_of(experts[0], net).s.C == C, NVDB_E_INVALID, "expert output count");
    for (int attempt = 0; attempt < 2; ++attempt) {
      NVDB_REQUIRE(cap < (1ull << 32), NVDB_E_INVALID, "too many routed pairs for the grouped decode");
      const size_t o_bs = (12 * cap + 255) & ~(size_t)255;
      const size_t o_ys = o_bs + ((4 * cap + 255) & ~(size_t)255);
      ws.big.ensure(o_ys + 32 * (size_t)C * (size_t)n);
      uint8_t* big = ws.big.p;
      float* bx = (float*)big;
      uint32_t* bslot = (uint32_t*)(big + o_bs);
      float* yslot = (float*)(big + o_ys);
      NVDB_HIP(hipMemcpyAsync(small, hs, small_bytes, hipMemcpyHostToDevice, st));
      moe_count(*tree, kind, g, tab, n_experts, cnt, cnt + n_experts, st);
      moe_plan(cnt, n_experts, (int)CH, cap, cs, start, flag, st);
      moe_route(*tree, kind, g, tab, dbox, n_experts, start, cursor, bx, bslot, cap, st);
      InferGroupLaunch M{};
      M.nets = gnets;
      M.n_nets = n_experts;
      M.chunk_start = cs;
      M.count = cnt;
      M.x = bx;
      M.slot = bslot;
      M.yslot = yslot;
      launch_infer_group(ks0, M, st);
      moe_blend(*tree, kind, g, tab, yslot, valued ? values_dev : nullptr,
                kind == MOE_VOXEL_SLOTS ? mask_dev : nullptr, kind == MOE_LEAF_SLOTS ? cls_dev : nullptr, st);
      NVDB_HIP(hipMemcpyAsync(back, flag, 8, hipMemcpyDeviceToHost, st));
      NVDB_HIP(hipStreamSynchronize(st));
      NVDB_REQUIRE(back[1] == 0, NVDB_E_INVALID, "items (voxels, slots or tiles) that no expert's widened box holds");
      if (back[0] == 0) return;
      std::vector<uint32_t> hc(E);
      NVDB_HIP(hipMemcpy(hc.data(), cnt, E * 4, hipMemcpyDeviceToHost));
      size_t need = 0;
      for (size_t k = 0; k < E; ++k) need += (hc[k] + CH - 1) / CH * CH;
      cap = need;
    }
    NVDB_REQUIRE(false, NVDB_E_DEVICE, "the routed pair count changed between two passes");
  }
  // small arrays in one allocation: lookup table, boxes, counts (+ the
  // uncovered voxels), bucket starts, cursors
  const size_t o_box = ((size_t)total * 4 + 255) & ~(size_t)255;
  const size_t o_cnt = o_box + ((E * sizeof(MoeBox) + 255) & ~(size_t)255);
  const size_t o_start = o_cnt + (((E + 1) * 4 + 255) & ~(size_t)255);
  const size_t o_cur = o_start + ((E * 4 + 255) & ~(size_t)255);
  MoeScratch& ws = moe_scratch();
  std::lock_guard<std::mutex> lock(ws.mu);
  StreamDrain drain{st};  // declared after the lock: runs before it is released
  ws.small.ensure(o_cur + E * 4);
  uint8_t* small = ws.small.p;
  int32_t* tab = (int32_t*)small;
  MoeBox* dbox = (MoeBox*)(small + o_box);
  uint32_t* cnt = (uint32_t*)(small + o_cnt);
  uint32_t* start = (uint32_t*)(small + o_start);
  uint32_t* cursor = (uint32_t*)(small + o_cur);
  NVDB_HIP(hipMemcpyAsync(tab, table.data(), (size_t)total * 4, hipMemcpyHostToDevice, st));
  NVDB_HIP(hipMemcpyAsync(dbox, box.data(), E * sizeof(MoeBox), hipMemcpyHostToDevice, st));
  NVDB_HIP(hipMemsetAsync(cnt, 0, (E + 1) * 4, st));
  NVDB_HIP(hipMemsetAsync(cursor, 0, E * 4, st));
  moe_count(*tree, kind, g, tab, n_experts, cnt, cnt + n_experts, st);
  std::vector<uint32_t> hc(E + 1);
  NVDB_HIP(hipMemcpyAsync(hc.data(), cnt, hc.size() * 4, hipMemcpyDeviceToHost, st));
  NVDB_HIP(hipStreamSynchronize(st));
  NVDB_REQUIRE(hc[E] == 0, NVDB_E_INVALID, "items (voxels, slots or tiles) that no expert's widened box holds");
  std::vector<uint32_t> hs(E);
  uint64_t pairs = 0;
  for (size_t k = 0; k < E; ++k) {
    hs[k] = (uint32_t)pairs;
    pairs += hc[k];
  }
  // per-pair coordinates, outputs (C each) and slots, and eight slots per item, in one allocation
  const size_t o_y = (12 * pairs + 255) & ~(size_t)255;
  const size_t o_bs = o_y + ((4 * (size_t)C * pairs + 255) & ~(size_t)255);
  const size_t o_ys = o_bs + ((4 * pairs + 255) & ~(size_t)255);
  ws.big.ensure(o_ys + 32 * (size_t)C * (size_t)n);
  uint8_t* big = ws.big.p;
  float* bx = (float*)big;
  float* y = (float*)(big + o_y);
  uint32_t* bslot = (uint32_t*)(big + o_bs);
  float* yslot = (float*)(big + o_ys);
  NVDB_HIP(hipMemcpyAsync(start, hs.data(), E * 4, hipMemcpyHostToDevice, st));
  moe_route(*tree, kind, g, tab, dbox, n_experts, start, cursor, bx, bslot, pairs, st);
  for (size_t k = 0; k < E; ++k) {
    if (hc[k] == 0) continue;
    const Net& N = net_of(experts[k], net);
    InferLaunch I{};
    I.net = net_view(N);
    base_spec(experts[k], &I.spec);
    I.spec.src = SRC_COORDS;
    I.spec.direct = 1;
    I.spec.coords = bx + 3 * (size_t)hs[k];
    I.spec.n = hc[k];
    I.out_kind = OUT_Y;
    I.y = y + (size_t)C * hs[k];
    launch_infer(N.ks, I, infer_grid(N.ks, hc[k]), st);
    query_scatter(y + (size_t)C * hs[k], bslot + hs[k], hc[k], cnt + k, valued ? experts[k]->d.value_scale : 1.f,
                  yslot, st, C);
  }
  moe_blend(*tree, kind, g, tab, yslot, valued ? values_dev : nullptr, slots ? mask_dev : nullptr,
            kind == MOE_LEAF_SLOTS ? cls_dev : nullptr, st);
  NVDB_HIP(hipStreamSynchronize(st));
}

extern "C" {

nvdb_status nvdb_decode_moe(const nvdb_model* const* experts, const int32_t* cells, int32_t n_experts,
                            const nvdb_subdomains* grid, const nvdb_tree* tree, float* values_dev, void* stream) {
  return guarded([&] {
    decode_moe_impl(experts, cells, n_experts, grid, tree, NVDB_NET_REGRESSOR, values_dev, nullptr, nullptr,
                    (hipStream_t)stream);
  });
}

nvdb_status nvdb_decode_moe_mask(const nvdb_model* const* experts, const int32_t* cells, int32_t n_experts,
                                 const nvdb_subdomains* grid, const nvdb_tree* tree, uint64_t* mask_dev,
                                 void* stream) {
  return guarded([&] {
    decode_moe_impl(experts, cells, n_experts, grid, tree, NVDB_NET_L0, nullptr, mask_dev, nullptr,
                    (hipStream_t)stream);
  });
}

nvdb_status nvdb_decode_moe_l1(const nvdb_model* const* experts, const int32_t* cells, int32_t n_experts,
                               const nvdb_subdomains* grid, const nvdb_tree* tree, uint8_t* classes_dev,
                               void* stream) {
  return guarded([&] {
    decode_moe_impl(experts, cells, n_experts, grid, tree, NVDB_NET_L1, nullptr, nullptr, classes_dev,
                    (hipStream_t)stream);
  });
}

nvdb_status nvdb_decode_moe_tiles(const nvdb_model* const* experts, const int32_t* cells, int32_t n_experts,
                                  const nvdb_subdomains* grid, const nvdb_tree* tree, float* tile_values_dev,
                                  void* stream) {
  return guarded([&] {
    decode_moe_impl(experts, cells, n_experts, grid, tree, NVDB_NET_TILE, tile_values_dev, nullptr, nullptr,
                    (hipStream_t)stream);
  });
}

}  // extern "C"

// Forward pass of one network over n samples given by spec (population indices
// of `tree`, or coordinates); no allocation.
static void forward_dev_impl(const nvdb_model* m, int32_t net, const Tree* tree, const SampleSpec& sp, float* y_dev,
                             hipStream_t st) {
  const Net& N = net_of(m, net);
  InferLaunch I{};
  I.net = net_view(N);
  I.spec = sp;
  I.tree = tree_view(tree);
  I.out_kind = OUT_Y;
  I.y = y_dev;
  launch_infer(N.ks, I, infer_grid(N.ks, sp.n), st);
  mark(m, st);
}

// Summed parameter gradient of sum_i gy_i . y(x_i) through the fused training
// kernel (activations recomputed), into grad_dev; workspace from the reservation.
static void backward_dev_impl(nvdb_model* m, int32_t net, const Tree* tree, SampleSpec sp, const float* gy_dev,
                              float* grad_dev, hipStream_t st) {
  Net& N = net_of(m, net);
  NVDB_REQUIRE(N.dev_n > 0 && sp.n <= N.dev_n, NVDB_E_STATE,
               "_dev workspace not reserved for this batch (nvdb_model_reserve_dev)");
  const int G = train_grid(sp.n, N.dev_G);
  TrainLaunch L{};
  L.G = G;
  TrainNet& tn = L.nets[0];
  tn.net = net_view(N);
  tn.tree = tree_view(tree);
  sp.loss = LOSS_EXTERNAL;
  sp.gy = gy_dev;
  sp.inv_n = 1.f;
  tn.spec = sp;
  tn.partial = N.dpart.p;
  tn.loss_partial = N.dlossp.p;
  launch_gather(tn.spec, tn.tree, N.dxt.p, st);
  tn.xt = N.dxt.p;
  launch_train(N.ks, L, 1, st);
  AdamLaunch AL{};
  AL.nets[0] = adam_view(N);
  AL.nets[0].partial = N.dpart.p;
  AL.nets[0].loss_partial = N.dlossp.p;
  AL.nets[0].G = G;
  AL.nets[0].grad_out = grad_dev;
  launch_reduce_adam(AL, N.s.nparams(), 1, st);
  mark(m, st);
}

// Sample spec of n population indices of network `net` on `tree`.
static SampleSpec index_spec(const nvdb_model* m, int32_t net, const Tree* tree, const uint32_t* idx, int64_t n) {
  NVDB_REQUIRE(tree != nullptr, NVDB_E_INVALID, "null tree");
  SampleSpec sp;
  base_spec(m, &sp);
  int64_t pop;
  sp.src = population_src(net, tree, &pop);
  NVDB_REQUIRE(pop > 0 && pop < (1ll << 32), NVDB_E_INVALID, "empty or oversized population");
  sp.npop = (uint32_t)pop;
  sp.idx = idx;
  sp.bad_idx = m->errw.p;
  sp.n = n;
  return sp;
}

static const Net& ready_net(const nvdb_model* m, int32_t net) {
  const Net& N = net_of(m, net);
  NVDB_REQUIRE(N.params_set && N.enc_set, NVDB_E_STATE, "parameters or encoding not set");
  return N;
}

extern "C" {

nvdb_status nvdb_model_reserve_dev(nvdb_model* m, int32_t net, int64_t max_n) {
  return guarded([&] {
    Net& N = net_of(m, net);
    NVDB_REQUIRE(max_n >= 1 && max_n <= (1 << 24), NVDB_E_INVALID, "max_n must be in 1..2^24");
    wait_model(m);
    const int G = train_grid(max_n, m->train_g > 0 ? m->train_g : DEFAULT_G);
    N.dev_n = 0;
    N.dpart.alloc((size_t)G * N.s.pstride());
    N.dlossp.alloc(G);
    N.dxt.alloc((size_t)max_n);
    N.dev_G = G;
    N.dev_n = max_n;
  });
}

nvdb_status nvdb_forward_dev(const nvdb_model* m, int32_t net, const nvdb_tree* tree, const uint32_t* idx_dev,
                             int64_t n, float* y_dev, void* stream) {
  return guarded([&] {
    ready_net(m, net);
    NVDB_REQUIRE(n >= 0 && n < (1ll << 31) && (n == 0 || (idx_dev && y_dev)), NVDB_E_INVALID, "bad buffers");
    if (n == 0) return;
    forward_dev_impl(m, net, tree, index_spec(m, net, tree, idx_dev, n), y_dev, (hipStream_t)stream);
  });
}

nvdb_status nvdb_backward_dev(nvdb_model* m, int32_t net, const nvdb_tree* tree, const uint32_t* idx_dev,
                              const float* gy_dev, int64_t n, float* grad_dev, void* stream) {
  return guarded([&] {
    ready_net(m, net);
    NVDB_REQUIRE(n >= 1 && idx_dev && gy_dev && grad_dev, NVDB_E_INVALID, "bad buffers");
    backward_dev_impl(m, net, tree, index_spec(m, net, tree, idx_dev, n), gy_dev, grad_dev, (hipStream_t)stream);
  });
}

nvdb_status nvdb_forward_coords_dev(const nvdb_model* m, int32_t net, const float* x_dev, int64_t n, float* y_dev,
                                    void* stream) {
  return guarded([&] {
    ready_net(m, net);
    NVDB_REQUIRE(n >= 0 && n < (1ll << 31) && (n == 0 || (x_dev && y_dev)), NVDB_E_INVALID, "bad buffers");
    if (n == 0) return;
    SampleSpec sp;
    base_spec(m, &sp);
    sp.src = SRC_COORDS;
    sp.direct = 1;
    sp.coords = x_dev;
    sp.n = n;
    forward_dev_impl(m, net, nullptr, sp, y_dev, (hipStream_t)stream);
  });
}

nvdb_status nvdb_backward_coords_dev(nvdb_model* m, int32_t net, const float* x_dev, const float* gy_dev, int64_t n,
                                     float* grad_dev, void* stream) {
  return guarded([&] {
    ready_net(m, net);
    NVDB_REQUIRE(n >= 1 && x_dev && gy_dev && grad_dev, NVDB_E_INVALID, "bad buffers");
    SampleSpec sp;
    base_spec(m, &sp);
    sp.src = SRC_COORDS;
    sp.coords = x_dev;
    sp.n = n;
    backward_dev_impl(m, net, nullptr, sp, gy_dev, grad_dev, (hipStream_t)stream);
  });
}

nvdb_status nvdb_model_set_params_dev(nvdb_model* m, int32_t net, const float* params_dev, int64_t n, void* stream) {
  return guarded([&] {
    Net& N = net_of(m, net);
    NVDB_REQUIRE(params_dev && n == N.s.nparams(), NVDB_E_INVALID, "parameter count mismatch");
    hipStream_t st = (hipStream_t)stream;
    NVDB_HIP(hipMemcpyAsync(N.theta.p, params_dev, n * 4, hipMemcpyDeviceToDevice, st));
    launch_write_shadow(adam_view(N), st);
    mark(m, st);
    N.params_set = true;
  });
}

nvdb_status nvdb_model_get_params_dev(const nvdb_model* m, int32_t net, float* params_dev, int64_t n, void* stream) {
  return guarded([&] {
    const Net& N = net_of(m, net);
    NVDB_REQUIRE(params_dev && n == N.s.nparams(), NVDB_E_INVALID, "parameter count mismatch");
    hipStream_t st = (hipStream_t)stream;
    NVDB_HIP(hipMemcpyAsync(params_dev, N.theta.p, n * 4, hipMemcpyDeviceToDevice, st));
    mark(m, st);
  });
}

nvdb_status nvdb_model_take_errors(nvdb_model* m, int64_t* n_bad_index) {
  return guarded([&] {
    NVDB_REQUIRE(m && n_bad_index, NVDB_E_INVALID, "null argument");
    *n_bad_index = take_bad_indices(m);
  });
}

nvdb_status nvdb_sample_indices_dev(uint64_t seed, int32_t stream_id, int64_t step, int64_t n_pop, int64_t batch,
                                    uint32_t* idx_dev, void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(n_pop > 0 && n_pop < (1ll << 32) && batch >= 0 && step >= 0 && stream_id >= 0, NVDB_E_INVALID,
                 "bad sampler arguments");
    NVDB_REQUIRE(batch == 0 || idx_dev, NVDB_E_INVALID, "null output");
    launch_sample(step_seed(seed, stream_id, step), (uint32_t)n_pop, batch, idx_dev, (hipStream_t)stream);
  });
}

}  // extern "C"

// ------------------------------------------------------------------ archive
// Byte image of a NeuralVDB: header, level-2 nodes (origin, child mask),
// level-1 nodes (origin; child and tile masks when stored explicitly), per
// network its shape, encoding matrix and 16-bit parameters, then the patch
// coordinates.  Little-endian, every section 4-byte aligned.
namespace {
struct ArchiveHeader {
  char magic[4];
  uint32_t version;
  uint32_t flags;    // bit 0: level-1 child / tile masks stored; bit 1: patches stored
  uint32_t storage;  // NVDB_STORE_F16 or NVDB_STORE_BF16
  int32_t precision;  // arithmetic the patches were taken with (the reader's)
  int32_t rule_kind;
  float rule_thr;
  float value_scale;
  int32_t domain_lo[3];
  int32_t domain_size;
  int32_t grid_origin[3];
  int32_t grid_dims[3];
  uint32_t nets_mask;
  uint32_t reserved;
  int64_t n_l2, n_l1, n_fp, n_fn, n_leaf;
};
static_assert(sizeof(ArchiveHeader) == 120, "archive header layout");
constexpr uint32_t ARCHIVE_VERSION = 1;
constexpr uint32_t AR_L1_MASKS = 1u, AR_PATCHES = 2u, AR_L0_MASKS = 4u;

int64_t pad4(int64_t n) { return (n + 3) & ~int64_t(3); }

struct Writer {
  uint8_t* buf;
  int64_t cap, pos = 0;
  void put(const void* p, int64_t n) {
    if (buf && pos + n <= cap) std::memcpy(buf + pos, p, (size_t)n);
    pos += n;
  }
  void pad() {
    static const uint8_t z[4] = {0, 0, 0, 0};
    put(z, pad4(pos) - pos);
  }
};
struct Reader {
  const uint8_t* buf;
  int64_t size, pos = 0;
  const uint8_t* take(int64_t n) {
    NVDB_REQUIRE(n >= 0 && pos + n <= size, NVDB_E_INVALID, "archive truncated");
    const uint8_t* p = buf + pos;
    pos += n;
    return p;
  }
  template <class T>
  T get() {
    T v;
    std::memcpy(&v, take(sizeof(T)), sizeof(T));
    return v;
  }
};

// A model holding the networks of `m` selected by nets_mask with their
// parameters rounded to 16 bits (the archive's content), in `precision`.
nvdb_model* rounded_model(const nvdb_model* m, int32_t nets_mask, int32_t storage, int32_t precision) {
  nvdb_model_desc d = m->d;
  d.precision = precision;
  for (int k = 0; k < NVDB_MAX_NETS; ++k) d.has_net[k] = (nets_mask >> k) & 1;
  nvdb_model* r = nullptr;
  nvdb_status st = nvdb_model_create(&d, &r);
  if (st != NVDB_OK) throw Error(st, g_err);
  try {
    for (int k = 0; k < NVDB_MAX_NETS; ++k) {
      if (!d.has_net[k]) continue;
      const Net& N = m->nets[k];
      const int64_t P = N.s.nparams();
      std::vector<uint16_t> p16((size_t)P);
      st = nvdb_model_get_params16(m, k, storage, p16.data(), P);
      if (st == NVDB_OK) st = nvdb_model_set_params16(r, k, storage, p16.data(), P);
      if (st != NVDB_OK) throw Error(st, g_err);
      std::vector<float> b(4 * (size_t)(N.s.KP / 2));
      NVDB_HIP(hipMemcpy(b.data(), N.benc.p, b.size() * 4, hipMemcpyDeviceToHost));
      std::vector<float> B3(3 * (size_t)N.d.n_freq);
      for (int i = 0; i < N.d.n_freq; ++i)
        for (int c = 0; c < 3; ++c) B3[3 * i + c] = b[4 * i + c];
      st = nvdb_model_set_encoding(r, k, B3.data(), N.d.n_freq);
      if (st != NVDB_OK) throw Error(st, g_err);
    }
  } catch (...) {
    delete r;
    throw;
  }
  return r;
}
}  // namespace

extern "C" {

nvdb_status nvdb_archive_write(const nvdb_model* m, const nvdb_tree* truth, const nvdb_archive_desc* ad, uint8_t* buf,
                               int64_t cap, int64_t* size, void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(m && truth && ad && size && cap >= 0 && (cap == 0 || buf), NVDB_E_INVALID, "null argument");
    NVDB_REQUIRE(ad->storage == NVDB_STORE_F16 || ad->storage == NVDB_STORE_BF16, NVDB_E_INVALID,
                 "unknown 16-bit format");
    const int32_t mask = ad->nets_mask;
    NVDB_REQUIRE(mask > 0 && mask < (1 << NVDB_MAX_NETS) && (mask & (1 << NVDB_NET_REGRESSOR)), NVDB_E_INVALID,
                 "an archive holds the regressor and optionally the classifiers");
    NVDB_REQUIRE(ad->explicit_l1 ? !(mask & (1 << NVDB_NET_L1)) : (mask & (1 << NVDB_NET_L1)) != 0, NVDB_E_INVALID,
                 "level-1 nodes are stored either as masks or as the level-1 classifier");
    NVDB_REQUIRE(!ad->explicit_l0 || (ad->explicit_l1 && !(mask & (1 << NVDB_NET_L0)) && !ad->patches),
                 NVDB_E_INVALID, "stored leaf masks need stored level-1 masks, no level-0 classifier and no patches");
    // voxel patches rebuild the reader's tree from voxels, which holds no tiles
    NVDB_REQUIRE(!(ad->patches && truth->n_tile > 0), NVDB_E_UNSUPPORTED,
                 "voxel patches of a tree with active tiles (store the leaf masks instead)");
    for (int k = 0; k < NVDB_MAX_NETS; ++k)
      if (mask & (1 << k)) {
        const Net& N = net_of(m, k);
        NVDB_REQUIRE(N.params_set && N.enc_set, NVDB_E_STATE, "parameters or encoding not set");
      }
    hipStream_t st = (hipStream_t)stream;
    wait_model(m);
    // the patches are taken against the topology the reader will decode: the same
    // 16-bit networks in the same arithmetic, from the stored upper levels
    std::vector<int32_t> fp, fn;
    if (ad->patches) {
      nvdb_model* r = rounded_model(m, mask, ad->storage, m->d.precision);
      nvdb_tree* upper = nullptr;
      nvdb_tree* pred = nullptr;
      try {
        if (ad->explicit_l1) {
          pred = decode_topology_impl(r, truth, false, st);
        } else {
          // the reader has no level-1 masks: decode from a copy of the upper levels without them
          upper = new nvdb_tree();
          upper->n_l1 = truth->n_l1;
          upper->n_l2 = truth->n_l2;
          upper->l2_origin = truth->l2_origin;
          upper->kind = truth->kind;
          upper->thr = truth->thr;
          std::memcpy(upper->origin, truth->origin, sizeof(upper->origin));
          std::memcpy(upper->dims, truth->dims, sizeof(upper->dims));
          const int64_t nl1 = std::max<int64_t>(truth->n_l1, 1);
          upper->l1_o.alloc(nl1);
          upper->l1_child.alloc(nl1 * 64);
          upper->l1_active.alloc(nl1 * 64);
          if (truth->n_l1)
            NVDB_HIP(hipMemcpyAsync(upper->l1_o.p, truth->l1_o.p, truth->n_l1 * sizeof(int4), hipMemcpyDeviceToDevice, st));
          NVDB_HIP(hipMemsetAsync(upper->l1_child.p, 0, nl1 * 64 * 8, st));
          NVDB_HIP(hipMemsetAsync(upper->l1_active.p, 0, nl1 * 64 * 8, st));
          pred = decode_topology_impl(r, upper, false, st);
        }
        int64_t nfp = 0, nfn = 0;
        NVDB_REQUIRE(truth->n_l1 == pred->n_l1, NVDB_E_STATE, "decoded tree lost level-1 nodes");
        nfp = topology_patches(*pred, *truth, nullptr, 0, st);
        nfn = topology_patches(*truth, *pred, nullptr, 0, st);
        DevBuf<int32_t> dfp, dfn;
        dfp.alloc(3 * std::max<int64_t>(nfp, 1));
        dfn.alloc(3 * std::max<int64_t>(nfn, 1));
        topology_patches(*pred, *truth, dfp.p, nfp, st);
        topology_patches(*truth, *pred, dfn.p, nfn, st);
        fp.resize(3 * (size_t)nfp);
        fn.resize(3 * (size_t)nfn);
        if (nfp) NVDB_HIP(hipMemcpy(fp.data(), dfp.p, 12 * (size_t)nfp, hipMemcpyDeviceToHost));
        if (nfn) NVDB_HIP(hipMemcpy(fn.data(), dfn.p, 12 * (size_t)nfn, hipMemcpyDeviceToHost));
      } catch (...) {
        delete pred;
        delete upper;
        delete r;
        throw;
      }
      delete pred;
      delete upper;
      delete r;
    }
    ArchiveHeader hd{};
    std::memcpy(hd.magic, "NVDB", 4);
    hd.version = ARCHIVE_VERSION;
    hd.flags = (ad->explicit_l1 ? AR_L1_MASKS : 0u) | (ad->patches ? AR_PATCHES : 0u) |
               (ad->explicit_l0 ? AR_L0_MASKS : 0u);
    hd.n_leaf = ad->explicit_l0 ? truth->n_leaf : 0;
    hd.storage = (uint32_t)ad->storage;
    hd.precision = m->d.precision;
    hd.rule_kind = truth->kind;
    hd.rule_thr = truth->thr;
    hd.value_scale = m->d.value_scale;
    for (int d = 0; d < 3; ++d) {
      hd.domain_lo[d] = m->d.domain_lo[d];
      hd.grid_origin[d] = truth->origin[d];
      hd.grid_dims[d] = truth->dims[d];
    }
    hd.domain_size = m->d.domain_size;
    hd.nets_mask = (uint32_t)mask;
    hd.n_l2 = truth->n_l2;
    hd.n_l1 = truth->n_l1;
    hd.n_fp = (int64_t)fp.size() / 3;
    hd.n_fn = (int64_t)fn.size() / 3;
    Writer w{buf, cap};
    w.put(&hd, sizeof(hd));
    // level 2
    std::vector<int32_t> l2o(3 * (size_t)truth->n_l2);
    std::vector<uint64_t> l2c(512 * (size_t)truth->n_l2);
    nvdb_status s2 = nvdb_tree_export_l2(truth, l2o.data(), l2c.data());
    if (s2 != NVDB_OK) throw Error(s2, g_err);
    for (int64_t i = 0; i < truth->n_l2; ++i) {
      w.put(&l2o[3 * i], 12);
      w.put(&l2c[512 * i], 4096);
    }
    // level 1
    if (truth->n_l1) {
      std::vector<int4> o((size_t)truth->n_l1);
      std::vector<uint64_t> c, a;
      NVDB_HIP(hipMemcpy(o.data(), truth->l1_o.p, truth->n_l1 * sizeof(int4), hipMemcpyDeviceToHost));
      if (ad->explicit_l1) {
        c.resize(64 * (size_t)truth->n_l1);
        a.resize(64 * (size_t)truth->n_l1);
        NVDB_HIP(hipMemcpy(c.data(), truth->l1_child.p, c.size() * 8, hipMemcpyDeviceToHost));
        NVDB_HIP(hipMemcpy(a.data(), truth->l1_active.p, a.size() * 8, hipMemcpyDeviceToHost));
      }
      for (int64_t i = 0; i < truth->n_l1; ++i) {
        const int32_t xyz[3] = {o[i].x, o[i].y, o[i].z};
        w.put(xyz, 12);
        if (ad->explicit_l1) {
          w.put(&c[64 * i], 512);
          w.put(&a[64 * i], 512);
        }
      }
    }
    // level 0
    if (ad->explicit_l0 && truth->n_leaf > 0) {
      std::vector<uint64_t> lm(8 * (size_t)truth->n_leaf);
      NVDB_HIP(hipMemcpy(lm.data(), truth->leaf_mask.p, lm.size() * 8, hipMemcpyDeviceToHost));
      w.put(lm.data(), 8 * (int64_t)lm.size());
    }
    // networks
    for (int k = 0; k < NVDB_MAX_NETS; ++k) {
      if (!(mask & (1 << k))) continue;
      const Net& N = m->nets[k];
      const int32_t desc[4] = {N.d.width, N.d.hidden, N.d.n_freq, N.d.n_out};
      w.put(desc, 16);
      w.put(&N.d.sin_freq, 4);
      std::vector<float> b(4 * (size_t)(N.s.KP / 2));
      NVDB_HIP(hipMemcpy(b.data(), N.benc.p, b.size() * 4, hipMemcpyDeviceToHost));
      for (int i = 0; i < N.d.n_freq; ++i) w.put(&b[4 * i], 12);
      const int64_t P = N.s.nparams();
      std::vector<uint16_t> p16((size_t)P);
      nvdb_status s3 = nvdb_model_get_params16(m, k, ad->storage, p16.data(), P);
      if (s3 != NVDB_OK) throw Error(s3, g_err);
      w.put(p16.data(), 2 * P);
      w.pad();
    }
    if (!fp.empty()) w.put(fp.data(), 4 * (int64_t)fp.size());
    if (!fn.empty()) w.put(fn.data(), 4 * (int64_t)fn.size());
    *size = w.pos;
    NVDB_REQUIRE(cap == 0 || w.pos <= cap, NVDB_E_INVALID, "archive buffer too small");
  });
}

nvdb_status nvdb_archive_decode(const uint8_t* buf, int64_t size, nvdb_tree** out, nvdb_archive_info* info,
                                void* stream) {
  return guarded([&] {
    NVDB_REQUIRE(buf && out && size >= 0, NVDB_E_INVALID, "null argument");
    *out = nullptr;
    hipStream_t st = (hipStream_t)stream;
    Reader r{buf, size};
    const ArchiveHeader hd = r.get<ArchiveHeader>();
    NVDB_REQUIRE(std::memcmp(hd.magic, "NVDB", 4) == 0 && hd.version == ARCHIVE_VERSION, NVDB_E_INVALID,
                 "not a NeuralVDB archive of this version");
    NVDB_REQUIRE((hd.flags & ~(AR_L1_MASKS | AR_PATCHES | AR_L0_MASKS)) == 0 && hd.nets_mask > 0 &&
                     hd.nets_mask < (1u << NVDB_MAX_NETS) && (hd.nets_mask & (1u << NVDB_NET_REGRESSOR)) &&
                     (hd.storage == NVDB_STORE_F16 || hd.storage == NVDB_STORE_BF16) &&
                     (hd.precision == NVDB_FP32 || hd.precision == NVDB_BF16) && hd.n_l2 >= 0 && hd.n_l1 >= 0 &&
                     hd.n_fp >= 0 && hd.n_fn >= 0 && hd.n_l1 < (1ll << 24) && hd.n_l2 < (1ll << 20) &&
                     hd.n_leaf >= 0 && hd.n_leaf <= 4096 * hd.n_l1,
                 NVDB_E_INVALID, "corrupt archive header");
    const bool explicit_l0 = hd.flags & AR_L0_MASKS;
    NVDB_REQUIRE(explicit_l0 ? ((hd.flags & AR_L1_MASKS) && !(hd.nets_mask & (1u << NVDB_NET_L0)) &&
                                !(hd.flags & AR_PATCHES))
                             : hd.n_leaf == 0,
                 NVDB_E_INVALID, "corrupt archive header");
    const bool explicit_l1 = hd.flags & AR_L1_MASKS;
    NVDB_REQUIRE(explicit_l1 == !(hd.nets_mask & (1u << NVDB_NET_L1)), NVDB_E_INVALID,
                 "archive must hold level-1 masks or a level-1 classifier, not both");
    // upper levels
    nvdb_tree* upper = new nvdb_tree();
    nvdb_model* model = nullptr;
    nvdb_tree* pred = nullptr;
    try {
      upper->kind = hd.rule_kind;
      upper->thr = hd.rule_thr;
      for (int d = 0; d < 3; ++d) {
        upper->origin[d] = hd.grid_origin[d];
        upper->dims[d] = hd.grid_dims[d];
      }
      upper->n_l2 = hd.n_l2;
      upper->n_l1 = hd.n_l1;
      upper->l2_origin.resize(3 * (size_t)hd.n_l2);
      for (int64_t i = 0; i < hd.n_l2; ++i) {
        std::memcpy(&upper->l2_origin[3 * i], r.take(12), 12);
        r.take(4096);  // child masks: implied by the level-1 origins
      }
      const int64_t nl1 = std::max<int64_t>(hd.n_l1, 1);
      std::vector<int4> o((size_t)nl1, int4{0, 0, 0, 0});
      std::vector<uint64_t> c(64 * (size_t)nl1, 0ull), a(64 * (size_t)nl1, 0ull);
      for (int64_t i = 0; i < hd.n_l1; ++i) {
        int32_t xyz[3];
        std::memcpy(xyz, r.take(12), 12);
        NVDB_REQUIRE((xyz[0] & 127) == 0 && (xyz[1] & 127) == 0 && (xyz[2] & 127) == 0, NVDB_E_INVALID,
                     "corrupt level-1 origin");
        o[i] = int4{xyz[0], xyz[1], xyz[2], 0};
        if (explicit_l1) {
          std::memcpy(&c[64 * i], r.take(512), 512);
          std::memcpy(&a[64 * i], r.take(512), 512);
        }
      }
      const uint8_t* leaf_masks = explicit_l0 ? r.take(64 * hd.n_leaf) : nullptr;
      upper->l1_o.alloc(nl1);
      upper->l1_child.alloc(64 * nl1);
      upper->l1_active.alloc(64 * nl1);
      NVDB_HIP(hipMemcpy(upper->l1_o.p, o.data(), nl1 * sizeof(int4), hipMemcpyHostToDevice));
      NVDB_HIP(hipMemcpy(upper->l1_child.p, c.data(), c.size() * 8, hipMemcpyHostToDevice));
      NVDB_HIP(hipMemcpy(upper->l1_active.p, a.data(), a.size() * 8, hipMemcpyHostToDevice));
      // networks
      nvdb_model_desc d{};
      d.precision = hd.precision;
      for (int k = 0; k < 3; ++k) d.domain_lo[k] = hd.domain_lo[k];
      d.domain_size = hd.domain_size;
      d.value_scale = hd.value_scale;
      struct Blob {
        const uint8_t* B;
        const uint8_t* p16;
        int64_t P;
      };
      Blob blobs[NVDB_MAX_NETS] = {};
      for (int k = 0; k < NVDB_MAX_NETS; ++k) {
        if (!(hd.nets_mask & (1u << k))) continue;
        int32_t desc[4];
        float sin_freq;
        std::memcpy(desc, r.take(16), 16);
        std::memcpy(&sin_freq, r.take(4), 4);
        NVDB_REQUIRE(desc[2] >= 1 && desc[2] <= 128 && desc[0] > 0 && desc[1] > 0 && desc[3] > 0, NVDB_E_INVALID,
                     "corrupt network shape");
        d.has_net[k] = 1;
        d.net[k] = nvdb_net_desc{desc[0], desc[1], desc[2], desc[3], sin_freq};
        blobs[k].B = r.take(12 * (int64_t)desc[2]);
        NetShape s{};
        s.K = 2 * desc[2];
        s.W = desc[0];
        s.H = desc[1];
        s.C = desc[3];
        blobs[k].P = s.nparams();
        blobs[k].p16 = r.take(pad4(2 * blobs[k].P));
      }
      nvdb_status s1 = nvdb_model_create(&d, &model);
      if (s1 != NVDB_OK) throw Error(s1, g_err);
      for (int k = 0; k < NVDB_MAX_NETS; ++k) {
        if (!d.has_net[k]) continue;
        std::vector<uint16_t> p16((size_t)blobs[k].P);
        std::memcpy(p16.data(), blobs[k].p16, 2 * (size_t)blobs[k].P);
        std::vector<float> B3(3 * (size_t)d.net[k].n_freq);
        std::memcpy(B3.data(), blobs[k].B, 12 * (size_t)d.net[k].n_freq);
        s1 = nvdb_model_set_params16(model, k, (int32_t)hd.storage, p16.data(), blobs[k].P);
        if (s1 == NVDB_OK) s1 = nvdb_model_set_encoding(model, k, B3.data(), d.net[k].n_freq);
        if (s1 != NVDB_OK) throw Error(s1, g_err);
      }
      const int32_t* fp = (const int32_t*)r.take(12 * hd.n_fp);
      const int32_t* fn = (const int32_t*)r.take(12 * hd.n_fn);
      NVDB_REQUIRE(r.pos == size, NVDB_E_INVALID, "trailing bytes after the archive");
      // the lower levels by inference (or from the stored leaf masks), then the patches
      DevBuf<uint64_t> lm;
      if (explicit_l0) {
        lm.alloc(std::max<int64_t>(8 * hd.n_leaf, 1));
        if (hd.n_leaf) NVDB_HIP(hipMemcpy(lm.p, leaf_masks, 64 * (size_t)hd.n_leaf, hipMemcpyHostToDevice));
      }
      pred = decode_topology_impl(model, upper, false, st, explicit_l0 ? lm.p : nullptr, hd.n_leaf);
      nvdb_tree* result = pred;
      if (hd.flags & AR_PATCHES) {
        DevBuf<int32_t> dfp, dfn;
        dfp.alloc(3 * std::max<int64_t>(hd.n_fp, 1));
        dfn.alloc(3 * std::max<int64_t>(hd.n_fn, 1));
        if (hd.n_fp) NVDB_HIP(hipMemcpy(dfp.p, fp, 12 * (size_t)hd.n_fp, hipMemcpyHostToDevice));
        if (hd.n_fn) NVDB_HIP(hipMemcpy(dfn.p, fn, 12 * (size_t)hd.n_fn, hipMemcpyHostToDevice));
        Tree* fixed = apply_patches(*pred, dfp.p, hd.n_fp, dfn.p, hd.n_fn, st);
        result = static_cast<nvdb_tree*>(fixed);
        delete pred;
        pred = nullptr;
        try {
          // values of the restored voxels from the regressor
          if (result->n_vox > 0) decode_impl(model, result, result->values.p, nullptr, false, st);
          NVDB_HIP(hipStreamSynchronize(st));
        } catch (...) {
          delete result;
          throw;
        }
      }
      if (info) {
        std::memset(info, 0, sizeof(*info));
        info->flags = (int32_t)hd.flags;
        info->nets_mask = (int32_t)hd.nets_mask;
        info->rule_kind = hd.rule_kind;
        info->rule_thr = hd.rule_thr;
        info->n_l2 = hd.n_l2;
        info->n_l1 = hd.n_l1;
        info->n_fp = hd.n_fp;
        info->n_fn = hd.n_fn;
        info->n_leaf = hd.n_leaf;
      }
      *out = result;
      pred = nullptr;
    } catch (...) {
      delete pred;
      delete model;
      delete upper;
      throw;
    }
    delete model;
    delete upper;
  });
}

}  // extern "C"
