// C ABI of the encoder library: model construction (weight conversion on the
// device), batch planning (variable-length packing of mixed-resolution
// images), workspace layout, kernel sequencing, optional HIP-graph replay,
// and the scoring entry point.  Declarations and contracts: include/vl.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <list>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/vl.h"
#include "kernels.hpp"
#include "plan.hpp"

using namespace vl;

namespace {

thread_local std::string g_last_error;

vl_status fail(vl_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

vl_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return VL_ERR_DEVICE;
}

#define VL_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call);  \
  } while (0)

static_assert(kNoAllocScratchBytes == VL_NOALLOC_SCRATCH_BYTES, "scratch size in vl.h");

struct Layer {
  const float *ln1_g, *ln1_b, *ln2_g, *ln2_b;
  const float *qkv_b, *o_b, *fc1_b, *fc2_b;
  const void *qkv_w, *o_w, *fc1_w, *fc2_w;          // f32, bf16 or e4m3 [out, in]
  const float *qkv_s, *o_s, *fc1_s, *fc2_s;         // per-row scales (e4m3 only)
  const uint8_t *qkv_x, *o_x, *fc1_x, *fc2_x;       // MXFP8 block scales [in/128][out][4]
  // LayerNorm folded into QKV / FC1 (BF16 and e4m3-weight models): c1 = W g,
  // c2 = W b + bias of LN1 -> QKV and LN2 -> FC1.
  const float *qkv_c1 = nullptr, *qkv_c2 = nullptr, *fc1_c1 = nullptr, *fc1_c2 = nullptr;
};

// Pinned host buffer holding a call's descriptors while its copy is pending.
struct Staging {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  void* host = nullptr;       // pinned descriptors captured by the graph's copy node
  hipEvent_t done = nullptr;  // recorded after each replay: the graph is idle once it fires
  uint64_t last_use = 0;      // replay clock, for least-recently-used eviction
};

constexpr size_t kMaxGraphs = 256;  // cached graphs per model

struct TimedLaunch {
  int op;
  hipEvent_t start, stop;
};

}  // namespace

struct vl_model {
  vl_config cfg;
  vl_precision prec;
  // Text models (vl_text_model_create): token table [vocab, D], position
  // table [ctx, D] (in `pos`), causal attention, last-token pooling.
  bool text = false;
  int vocab = 0, ctx = 0;
  const float* tok_emb = nullptr;
  int device = 0;
  int D, F, heads, hd, L, P, Pd, g0, Kpe, Kpad;
  char* wmem = nullptr;
  size_t wbytes = 0;
  const void* patch_w = nullptr;  // folded [D, Kpad], f32 or bf16
  const float *patch_b, *cls, *pos, *lnf_g, *lnf_b, *proj;
  // MAP pooling head (VL_POOL_MAP): projected probe q = probe W_q^T + b_q
  // (FP32, computed once), K/V projection [2D, D] (BF16, FP32 for VL_FP32),
  // and the FP32 output projection, LayerNorm and MLP.
  const float *map_q = nullptr, *map_kv_b = nullptr, *map_o_w = nullptr, *map_o_b = nullptr;
  const float *map_ln_g = nullptr, *map_ln_b = nullptr, *map_fc1_w = nullptr, *map_fc1_b = nullptr;
  const float *map_fc2_w = nullptr, *map_fc2_b = nullptr;
  const float *map_probe = nullptr, *map_q_w = nullptr;   // for the training backward
  const void* map_kv_w = nullptr;
  std::vector<Layer> layers;
  bool use_graphs = false;
  std::mutex mu;
  std::vector<Staging> ring;
  size_t ring_pos = 0;
  std::unordered_map<std::string, GraphEntry> graphs;
  uint64_t graph_clock = 0;
  int64_t graph_captures = 0, graph_replays = 0;   // since creation
  // One event per stream the model has been used on, recorded at the end of
  // every call on it: waiting for all of them waits for all of the model's
  // enqueued work, without synchronising the device.
  std::unordered_map<hipStream_t, hipEvent_t> last_use;
  bool timing = false;
  std::vector<TimedLaunch> timed;      // recorded, not yet harvested
  std::vector<hipEvent_t> free_events;
  double op_ms[VL_N_OPS] = {};
  int64_t op_launches[VL_N_OPS] = {};
  hipStream_t capture = nullptr;  // private stream graphs are captured on
  // Two-part batches (off by default): the second part runs on this stream,
  // forked from and joined back into the caller's stream with the two events.
  bool split = false;
  // LayerNorm folded into the neighbouring GEMMs (BF16 and e4m3-weight
  // models; VL_OPT_FUSED_LN, off by default: on MI355X the extra epilogue
  // output costs the GEMMs more than the standalone LayerNorms take).
  bool fused_ln = false;
  // K/V-resident attention for images of 129 .. 640 tokens (BF16 attention,
  // head width 64, not causal; VL_OPT_ATTN_RESIDENT, on by default).
  bool attn_resident = true;
  // Graph replay per capacity bucket where the model supports it
  // (VL_OPT_GRAPH_BUCKETS, on by default).
  bool graph_buckets = true;
  bool kmajor_wgrad = true;   // BF16 weight gradients from token-major operands
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // Training backward: ordering between the caller's stream and the side
  // stream that runs the weight-gradient GEMMs (see run_backward).
  hipEvent_t tev[10] = {};
  // BF16 training backward: every block's transposed weights (W_qkv^T
  // [D, 3D], W_o^T [D, D], W_1^T [D, F], W_2^T [F, D]), formed by the first
  // backward call and kept, since a model's weights never change after
  // creation; wT_ev marks the end of that fill.
  char* wT = nullptr;
  hipEvent_t wT_ev = nullptr;
  int32_t tuning[VL_N_GEMM_OPS][VL_N_M_BUCKETS];
  // The last vl_encode_images_train call (workspace, pixels, shapes): the
  // backward pass must be given the same, since it reads what that forward
  // kept in the workspace.
  std::string train_key;
};

namespace {

bool config_ok(const vl_config* c, std::string* why) {
  if (!c) { *why = "cfg is NULL"; return false; }
  if (c->patch < 1 || c->width <= 0 || c->layers < 0 || c->heads <= 0 || c->mlp <= 0 ||
      c->proj_dim <= 0 || c->base_grid < 1) {
    *why = "non-positive dimension in cfg";
    return false;
  }
  if (c->width % c->heads) { *why = "width % heads != 0"; return false; }
  if (c->width % 128 || c->mlp % 128) { *why = "width and mlp must be multiples of 128"; return false; }
  if (c->proj_dim % 4) { *why = "proj_dim must be a multiple of 4"; return false; }
  if (c->proj_dim > 1024) { *why = "proj_dim must be <= 1024"; return false; }
  if (!(c->ln_eps >= 0.f)) { *why = "ln_eps must be >= 0"; return false; }
  if (c->channels < 1 || c->channels > 4) { *why = "channels must be 1..4"; return false; }
  if (c->pool != VL_POOL_CLS && c->pool != VL_POOL_MAP) { *why = "unknown pool"; return false; }
  for (int i = 0; i < c->channels; ++i)
    if (!(c->chan_std[i] > 0.f)) { *why = "chan_std must be > 0"; return false; }
  return true;
}

bool text_config_ok(const vl_text_config* c, std::string* why) {
  if (!c) { *why = "cfg is NULL"; return false; }
  if (c->vocab < 1 || c->ctx < 1 || c->width <= 0 || c->layers < 0 || c->heads <= 0 ||
      c->mlp <= 0 || c->proj_dim <= 0) {
    *why = "non-positive dimension in cfg";
    return false;
  }
  if (c->ctx > 1024) { *why = "ctx must be <= 1024"; return false; }
  if (c->width % c->heads) { *why = "width % heads != 0"; return false; }
  if (c->width % 128 || c->mlp % 128) { *why = "width and mlp must be multiples of 128"; return false; }
  if (c->proj_dim % 4 || c->proj_dim > 1024) { *why = "proj_dim must be a multiple of 4, <= 1024"; return false; }
  if (!(c->ln_eps >= 0.f)) { *why = "ln_eps must be >= 0"; return false; }
  return true;
}

size_t text_weights_count(const vl_text_config& c) {
  const size_t D = c.width, F = c.mlp;
  size_t n = (size_t)c.vocab * D + (size_t)c.ctx * D;
  n += (size_t)c.layers * (2 * D + 3 * D * D + 3 * D + D * D + D + 2 * D + F * D + F + D * F + D);
  n += 2 * D + (size_t)c.proj_dim * D;
  return n;
}

size_t weights_count(const vl_config& c) {
  const size_t D = c.width, F = c.mlp, P = c.patch, g = c.base_grid;
  size_t n = D * c.channels * P * P + D + D + (1 + g * g) * D;
  n += (size_t)c.layers * (2 * D + 3 * D * D + 3 * D + D * D + D + 2 * D + F * D + F + D * F + D);
  n += 2 * D + (size_t)c.proj_dim * D;
  if (c.pool == VL_POOL_MAP) n += D + (D * D + D) + (2 * D * D + 2 * D) + (D * D + D) + 2 * D +
                                  (F * D + F) + (D * F + D);
  return n;
}

// ----------------------------------------------------------------- planning
// The planner itself is host-only code (plan.hpp); these give it the
// model's view.
PlanModel plan_model(const vl_model* m) {
  PlanModel pm;
  pm.text = m->text;
  pm.split = m->split && m->prec != VL_FP32;
  pm.resident = m->attn_resident && m->prec != VL_FP32 && m->hd == 64 && !m->text;
  pm.map_pool = !m->text && m->cfg.pool == VL_POOL_MAP;
  pm.fold_buffers = m->prec == VL_BF16 || m->prec == VL_FP8W_BF16A;
  pm.es = m->prec == VL_FP32 ? 4 : 2;
  pm.D = m->D; pm.F = m->F; pm.Kpad = m->Kpad; pm.Pd = m->Pd;
  pm.P = m->P; pm.channels = m->cfg.channels; pm.ctx = m->ctx;
  return pm;
}

bool make_plan(const vl_model* m, int32_t n, const int32_t* hs, const int32_t* ws, Plan* p,
               std::string* why, bool one_part = false, bool bucketed = false) {
  return vl::make_plan(plan_model(m), n, hs, ws, p, why, one_part, bucketed);
}

bool make_text_plan(const vl_model* m, int32_t n, const int32_t* lens, Plan* p,
                    std::string* why) {
  return vl::make_text_plan(plan_model(m), n, lens, p, why);
}

// Whether the model's encode calls plan for capacity buckets: graph replay
// on, and a kernel sequence whose launches all read live counts on the
// device (BF16 or e4m3-weight image models with class-token pooling and
// standalone LayerNorms).
bool bucket_mode(const vl_model* m) {
  return m->use_graphs && m->graph_buckets && !m->text &&
         (m->prec == VL_BF16 || m->prec == VL_FP8W_BF16A) && m->cfg.pool == VL_POOL_CLS &&
         !m->fused_ln;
}

// Async copy of `bytes` host bytes to dst through the next pinned buffer of
// a staging ring; a buffer is reused once the copy it last served is done.
vl_status stage_copy(std::vector<Staging>& ring, size_t& pos, const void* src, size_t bytes,
                     void* dst, hipStream_t s) {
  Staging& st = ring[pos];
  pos = (pos + 1) % ring.size();
  if (st.pending) {
    VL_HIP(hipEventSynchronize(st.ev));
    st.pending = false;
  }
  if (st.cap < bytes) {
    if (st.host) VL_HIP(hipHostFree(st.host));
    st.host = nullptr;
    st.cap = 0;
    const size_t cap = std::max<size_t>(bytes, 16384);
    VL_HIP(hipHostMalloc(&st.host, cap, hipHostMallocDefault));
    st.cap = cap;
  }
  if (!st.ev) VL_HIP(hipEventCreateWithFlags(&st.ev, hipEventDisableTiming));
  std::memcpy(st.host, src, bytes);
  VL_HIP(hipMemcpyAsync(dst, st.host, bytes, hipMemcpyHostToDevice, s));
  VL_HIP(hipEventRecord(st.ev, s));
  st.pending = true;
  return VL_OK;
}

// Upload the plan's descriptors with an async copy from pinned memory.
vl_status stage_descriptors(vl_model* m, const Plan& p, void* dst, hipStream_t s) {
  return stage_copy(m->ring, m->ring_pos, p.desc.data(), p.desc_bytes, dst, s);
}

enum { T_PATCH = 0, T_LN, T_QKV, T_ATTN, T_OPROJ, T_FC1, T_FC2, T_POOL };

int m_bucket(int M) {
  int b = 0;
  while ((2 << b) <= M && b < VL_N_M_BUCKETS - 1) ++b;
  return b;
}

// Tile configuration for GEMM operation op (0 patch .. 4 fc2) at M rows.
int gemm_cfg_for(const vl_model* m, int op, int M) {
  return m->tuning[op][m_bucket(M)];
}

hipError_t take_event(vl_model* m, hipEvent_t* ev) {
  if (!m->free_events.empty()) {
    *ev = m->free_events.back();
    m->free_events.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(ev);
}

// Brackets the launches of one operation with events when timing is on.
struct OpScope {
  vl_model* m;
  hipStream_t s;
  TimedLaunch t{};
  bool on;
  hipError_t err = hipSuccess;
  OpScope(vl_model* m_, int op, hipStream_t s_) : m(m_), s(s_), on(m_->timing) {
    if (!on) return;
    t.op = op;
    if ((err = take_event(m, &t.start)) != hipSuccess) return;
    if ((err = take_event(m, &t.stop)) != hipSuccess) return;
    err = hipEventRecord(t.start, s);
  }
  hipError_t close() {
    if (!on || err != hipSuccess) return err;
    err = hipEventRecord(t.stop, s);
    if (err == hipSuccess) m->timed.push_back(t);
    return err;
  }
};

#define VL_TIMED(op, ...)                                 \
  do {                                                    \
    OpScope sc_(m, op, s);                                \
    if (sc_.err != hipSuccess) return hip_fail(sc_.err, "timing event"); \
    __VA_ARGS__;                                          \
    VL_HIP(sc_.close());                                  \
  } while (0)

// The kernel sequence of one part of an encode call.
vl_status run_part(vl_model* m, const Part& p, const void* in, float* emb, char* ws,
                   hipStream_t s, hipEvent_t after_first_qkv = nullptr) {
  const bool f32 = m->prec == VL_FP32;
  const bool fp8 = m->prec == VL_FP8W_BF16A;
  const bool mx = m->prec == VL_MXFP8;
  const ImgDesc* d_imgs = reinterpret_cast<const ImgDesc*>(ws + p.off_imgs);
  const AttnItem* d_items = reinterpret_cast<const AttnItem*>(ws + p.off_items);
  const int* d_res = reinterpret_cast<const int*>(ws + p.off_res);
  int2* tok = reinterpret_cast<int2*>(ws + p.off_tok);
  float* X = reinterpret_cast<float*>(ws + p.off_X);
  void* Y = ws + p.off_Y;
  void* QH = ws + p.off_QH;
  // Launch sizes: the part's counts, or its bucket's capacities with the
  // live counts in the device record bc.
  const int T = p.T_cap, D = m->D, F = m->F;
  const BatchCounts* bc = p.bucketed ? reinterpret_cast<const BatchCounts*>(ws + p.off_bc) : nullptr;
  const int32_t* m_dev = bc ? &bc->T : nullptr;
  const float eps = m->cfg.ln_eps;

  EpiArgs pe;
  pe.bias = m->patch_b;
  pe.out = X;
  pe.ldo = D;
  pe.tok_info = tok;
  pe.imgs = d_imgs;
  pe.cls = m->cls;
  pe.pos = m->pos;
  pe.base_grid = m->g0;
  pe.m_dev = m_dev;
  if (m->text)
    VL_TIMED(T_PATCH, VL_HIP(text_embed(static_cast<const int32_t*>(in), d_imgs, p.n, p.max_ntok,
                                        m->tok_emb, m->pos, m->vocab, D, X, tok, s)));
  else VL_TIMED(T_PATCH, {
    VL_HIP(im2col(static_cast<const float*>(in), d_imgs, p.n_cap, p.ntok_cap, m->cfg.channels,
                  m->P, m->Kpad, QH, !f32, tok, s, bc));
    if (f32)
      VL_HIP(gemm_f32(static_cast<const float*>(QH), m->Kpad,
                      static_cast<const float*>(m->patch_w), m->Kpad, T, D, m->Kpad, OP_PATCH,
                      pe, s));
    else
      VL_HIP(gemm_bf16(static_cast<const bf16_t*>(QH), m->Kpad, m->patch_w, m->Kpad, false, T,
                       D, m->Kpad, OP_PATCH, gemm_cfg_for(m, 0, T), pe, s));
  });

  // LayerNorm folding (BF16 / e4m3 weights): the GEMMs read u = bf16(x g)
  // and the row statistics; the residual epilogues produce both for the
  // next LayerNorm, the first block's come from one folding pass.
  const bool fold = !f32 && !mx && m->fused_ln && !m->layers.empty();
  bf16_t* U = reinterpret_cast<bf16_t*>(ws + p.off_U);
  float* PS = reinterpret_cast<float*>(ws + p.off_PS);
  float* RS = reinterpret_cast<float*>(ws + p.off_RS);
  if (fold)
    VL_TIMED(T_LN, VL_HIP(ln_fold_rows(X, m->layers[0].ln1_g, eps, U, RS, T, D, s)));
  for (size_t li = 0; li < m->layers.size(); ++li) {
    const Layer& ly = m->layers[li];
    if (fold) {
      const Layer* nx = li + 1 < m->layers.size() ? &m->layers[li + 1] : nullptr;
      EpiArgs e1; e1.wscale = ly.qkv_s; e1.out = QH; e1.ldo = 3 * D;
      e1.row_stats = RS; e1.c1 = ly.qkv_c1; e1.c2 = ly.qkv_c2;
      EpiArgs e2; e2.bias = ly.o_b; e2.wscale = ly.o_s; e2.out = X; e2.ldo = D;
      e2.u_out = U; e2.u_gamma = ly.ln2_g; e2.part_stats = PS;
      EpiArgs e3; e3.wscale = ly.fc1_s; e3.out = QH; e3.ldo = F;
      e3.row_stats = RS; e3.c1 = ly.fc1_c1; e3.c2 = ly.fc1_c2;
      EpiArgs e4; e4.bias = ly.fc2_b; e4.wscale = ly.fc2_s; e4.out = X; e4.ldo = D;
      if (nx) { e4.u_out = U; e4.u_gamma = nx->ln1_g; e4.part_stats = PS; }
      const bf16_t* qh = static_cast<const bf16_t*>(QH);
      VL_TIMED(T_QKV, VL_HIP(gemm_bf16(U, D, ly.qkv_w, D, fp8, T, 3 * D, D, OP_QKV,
                                       gemm_cfg_for(m, 1, T), e1, s)));
      if (after_first_qkv && li == 0) VL_HIP(hipEventRecord(after_first_qkv, s));
      VL_TIMED(T_ATTN, {
        VL_HIP(attention_bf16(qh, static_cast<bf16_t*>(Y), d_imgs, d_items, p.n_items, m->heads,
                              m->hd, m->text, s));
        VL_HIP(attention_bf16_resident(qh, Y, nullptr, false, T, d_imgs, d_res, p.n_res,
                                       p.res_tiles, m->heads, m->hd, s));
      });
      VL_TIMED(T_OPROJ, VL_HIP(gemm_bf16(static_cast<const bf16_t*>(Y), D, ly.o_w, D, fp8, T, D,
                                         D, OP_OPROJ, gemm_cfg_for(m, 2, T), e2, s)));
      VL_TIMED(T_LN, VL_HIP(ln_stats_from_parts(PS, T, D, eps, RS, s)));
      VL_TIMED(T_FC1, VL_HIP(gemm_bf16(U, D, ly.fc1_w, D, fp8, T, F, D, OP_FC1,
                                       gemm_cfg_for(m, 3, T), e3, s)));
      VL_TIMED(T_FC2, VL_HIP(gemm_bf16(qh, F, ly.fc2_w, F, fp8, T, D, F, OP_FC2,
                                       gemm_cfg_for(m, 4, T), e4, s)));
      if (nx) VL_TIMED(T_LN, VL_HIP(ln_stats_from_parts(PS, T, D, eps, RS, s)));
      continue;
    }
    if (mx)
      VL_TIMED(T_LN, VL_HIP(layernorm_rows_mx(X, ly.ln1_g, ly.ln1_b, eps, static_cast<uint8_t*>(Y),
                                              static_cast<uint8_t*>(Y) + (size_t)T * D, T, D, s)));
    else
      VL_TIMED(T_LN, VL_HIP(layernorm_rows(X, ly.ln1_g, ly.ln1_b, eps, Y, !f32, T, D, s, bc)));
    EpiArgs e1;
    e1.bias = ly.qkv_b; e1.wscale = ly.qkv_s; e1.out = QH; e1.ldo = 3 * D; e1.m_dev = m_dev;
    EpiArgs e2;
    e2.bias = ly.o_b; e2.wscale = ly.o_s; e2.out = X; e2.ldo = D; e2.m_dev = m_dev;
    EpiArgs e3;
    e3.bias = ly.fc1_b; e3.wscale = ly.fc1_s; e3.out = QH; e3.ldo = F; e3.m_dev = m_dev;
    EpiArgs e4;
    e4.bias = ly.fc2_b; e4.wscale = ly.fc2_s; e4.out = X; e4.ldo = D; e4.m_dev = m_dev;
    if (f32) {
      const float* y = static_cast<const float*>(Y);
      const float* qh = static_cast<const float*>(QH);
      VL_TIMED(T_QKV, VL_HIP(gemm_f32(y, D, static_cast<const float*>(ly.qkv_w), D, T, 3 * D, D,
                                      OP_QKV, e1, s)));
      VL_TIMED(T_ATTN, VL_HIP(attention_f32(qh, static_cast<float*>(Y), d_imgs, d_items,
                                            p.n_items, m->heads, m->hd, m->text, s)));
      VL_TIMED(T_OPROJ, VL_HIP(gemm_f32(y, D, static_cast<const float*>(ly.o_w), D, T, D, D,
                                        OP_OPROJ, e2, s)));
      VL_TIMED(T_LN, VL_HIP(layernorm_rows(X, ly.ln2_g, ly.ln2_b, eps, Y, false, T, D, s)));
      VL_TIMED(T_FC1, VL_HIP(gemm_f32(y, D, static_cast<const float*>(ly.fc1_w), D, T, F, D,
                                      OP_FC1, e3, s)));
      VL_TIMED(T_FC2, VL_HIP(gemm_f32(qh, F, static_cast<const float*>(ly.fc2_w), F, T, D, F,
                                      OP_FC2, e4, s)));
    } else if (mx) {
      // MXFP8 GEMM operands: codes then E8M0 scales in the Y and QH regions
      // (LN / attention output in Y; GELU output in QH after attention has
      // consumed the QKV rows there).
      uint8_t* y8 = static_cast<uint8_t*>(Y);
      uint8_t* ys = y8 + (size_t)T * D;
      uint8_t* h8 = static_cast<uint8_t*>(QH);
      uint8_t* hs = h8 + (size_t)T * F;
      const uint8_t* w8[4] = {static_cast<const uint8_t*>(ly.qkv_w), static_cast<const uint8_t*>(ly.o_w),
                              static_cast<const uint8_t*>(ly.fc1_w), static_cast<const uint8_t*>(ly.fc2_w)};
      e3.out = h8; e3.out_scale = hs; e3.scale_rows = T;
      VL_TIMED(T_QKV, VL_HIP(gemm_mx(y8, ys, w8[0], ly.qkv_x, T, 3 * D, D, OP_QKV,
                                     gemm_cfg_for(m, 1, T), e1, s)));
      if (after_first_qkv && &ly == &m->layers[0]) VL_HIP(hipEventRecord(after_first_qkv, s));
      VL_TIMED(T_ATTN, {
        VL_HIP(attention_bf16_mx(static_cast<const bf16_t*>(QH), y8, ys, T, d_imgs, d_items,
                                 p.n_items, m->heads, m->hd, m->text, s));
        VL_HIP(attention_bf16_resident(static_cast<const bf16_t*>(QH), y8, ys, true, T, d_imgs,
                                       d_res, p.n_res, p.res_tiles, m->heads, m->hd, s));
      });
      VL_TIMED(T_OPROJ, VL_HIP(gemm_mx(y8, ys, w8[1], ly.o_x, T, D, D, OP_OPROJ,
                                       gemm_cfg_for(m, 2, T), e2, s)));
      VL_TIMED(T_LN, VL_HIP(layernorm_rows_mx(X, ly.ln2_g, ly.ln2_b, eps, y8, ys, T, D, s)));
      VL_TIMED(T_FC1, VL_HIP(gemm_mx(y8, ys, w8[2], ly.fc1_x, T, F, D, OP_FC1,
                                     gemm_cfg_for(m, 3, T), e3, s)));
      VL_TIMED(T_FC2, VL_HIP(gemm_mx(h8, hs, w8[3], ly.fc2_x, T, D, F, OP_FC2,
                                     gemm_cfg_for(m, 4, T), e4, s)));
    } else {
      const bf16_t* y = static_cast<const bf16_t*>(Y);
      const bf16_t* qh = static_cast<const bf16_t*>(QH);
      VL_TIMED(T_QKV, VL_HIP(gemm_bf16(y, D, ly.qkv_w, D, fp8, T, 3 * D, D, OP_QKV,
                                       gemm_cfg_for(m, 1, T), e1, s)));
      if (after_first_qkv && &ly == &m->layers[0]) VL_HIP(hipEventRecord(after_first_qkv, s));
      VL_TIMED(T_ATTN, {
        VL_HIP(attention_bf16(qh, static_cast<bf16_t*>(Y), d_imgs, d_items, p.items_cap,
                              m->heads, m->hd, m->text, s, bc));
        VL_HIP(attention_bf16_resident(qh, Y, nullptr, false, T, d_imgs, d_res, p.res_cap,
                                       p.res_class, m->heads, m->hd, s, bc));
      });
      VL_TIMED(T_OPROJ, VL_HIP(gemm_bf16(y, D, ly.o_w, D, fp8, T, D, D, OP_OPROJ,
                                         gemm_cfg_for(m, 2, T), e2, s)));
      VL_TIMED(T_LN, VL_HIP(layernorm_rows(X, ly.ln2_g, ly.ln2_b, eps, Y, true, T, D, s, bc)));
      VL_TIMED(T_FC1, VL_HIP(gemm_bf16(y, D, ly.fc1_w, D, fp8, T, F, D, OP_FC1,
                                       gemm_cfg_for(m, 3, T), e3, s)));
      VL_TIMED(T_FC2, VL_HIP(gemm_bf16(qh, F, ly.fc2_w, F, fp8, T, D, F, OP_FC2,
                                       gemm_cfg_for(m, 4, T), e4, s)));
    }
  }
  if (!m->text && m->cfg.pool == VL_POOL_MAP) {
    // MAP head: LN_f on every token -> K/V projection -> probe attention ->
    // output projection -> x + MLP(LN(x)) -> projection -> L2.
    float* mo = reinterpret_cast<float*>(ws + p.off_map);
    float* mx1 = mo + (size_t)p.n * D;
    float* my = mx1 + (size_t)p.n * D;
    float* mh = my + (size_t)p.n * D;
    float* e = reinterpret_cast<float*>(ws + p.off_E);
    VL_TIMED(T_POOL, {
      VL_HIP(layernorm_rows(X, m->lnf_g, m->lnf_b, eps, Y, !f32, T, D, s));
      EpiArgs ekv;
      ekv.bias = m->map_kv_b; ekv.out = QH; ekv.ldo = 2 * D;
      if (f32)
        VL_HIP(gemm_f32(static_cast<const float*>(Y), D, static_cast<const float*>(m->map_kv_w), D,
                        T, 2 * D, D, OP_QKV, ekv, s));
      else
        VL_HIP(gemm_bf16(static_cast<const bf16_t*>(Y), D, m->map_kv_w, D, false, T, 2 * D, D,
                         OP_QKV, -1, ekv, s));
      VL_HIP(map_attention(QH, !f32, m->map_q, d_imgs, p.n, m->heads, m->hd, mo, s));
      EpiArgs e1; e1.bias = m->map_o_b; e1.out = mx1; e1.ldo = D;
      VL_HIP(gemm_f32_rows(mo, D, m->map_o_w, D, p.n, D, D, OP_QKV, e1, s));
      VL_HIP(layernorm_rows(mx1, m->map_ln_g, m->map_ln_b, eps, my, false, p.n, D, s));
      EpiArgs e2; e2.bias = m->map_fc1_b; e2.out = mh; e2.ldo = F;
      VL_HIP(gemm_f32_rows(my, D, m->map_fc1_w, D, p.n, F, D, OP_FC1, e2, s));
      EpiArgs e3; e3.bias = m->map_fc2_b; e3.out = mx1; e3.ldo = D;
      VL_HIP(gemm_f32_rows(mh, F, m->map_fc2_w, F, p.n, D, F, OP_FC2, e3, s));
      EpiArgs e4; e4.out = e; e4.ldo = m->Pd;
      VL_HIP(gemm_f32_rows(mx1, D, m->proj, D, p.n, m->Pd, D, OP_LOGITS, e4, s));
      VL_HIP(l2_normalise_rows(e, emb + (size_t)p.i0 * m->Pd, p.n, m->Pd, s));
    });
    return VL_OK;
  }
  // The QKV region is free after the last block and holds the n x D pooled
  // rows (it is at least 3 x T x D x 2 bytes and T >= n).
  VL_TIMED(T_POOL, VL_HIP(pool_project(X, d_imgs, p.n_cap, m->lnf_g, m->lnf_b, eps, m->proj, D,
                                        m->Pd, m->text, static_cast<float*>(QH),
                                        reinterpret_cast<float*>(ws + p.off_E),
                                        emb + (size_t)p.i0 * m->Pd, s, bc)));
  return VL_OK;
}

// The kernel sequence of one encode call: a single part on the caller's
// stream, or two parts on the caller's stream and the model's side stream,
// forked after everything already on the caller's stream (the descriptor
// upload) and joined back before the call returns.  The two parts then
// overlap one another's tile-round tails, epilogue store bursts and
// non-MFMA phases.
vl_status run_encoder(vl_model* m, const Plan& p, const void* pix, float* emb, char* ws,
                      hipStream_t s) {
  if (p.parts.size() == 1) return run_part(m, p.parts[0], pix, emb, ws, s);
  if (!m->side) VL_HIP(hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking));
  if (!m->ev_fork) VL_HIP(hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming));
  if (!m->ev_join) VL_HIP(hipEventCreateWithFlags(&m->ev_join, hipEventDisableTiming));
  // The second part starts once the first has finished its first QKV GEMM,
  // so the two sequences run about one operation out of phase.
  vl_status st = run_part(m, p.parts[0], pix, emb, ws, s, m->layers.empty() ? nullptr : m->ev_fork);
  if (m->layers.empty()) VL_HIP(hipEventRecord(m->ev_fork, s));
  VL_HIP(hipStreamWaitEvent(m->side, m->ev_fork, 0));
  vl_status st2 = run_part(m, p.parts[1], pix, emb, ws, m->side);
  // Join even after an enqueue error, so a capture still ends cleanly.
  VL_HIP(hipEventRecord(m->ev_join, m->side));
  VL_HIP(hipStreamWaitEvent(s, m->ev_join, 0));
  return st != VL_OK ? st : st2;
}

// Graph cache key.  A bucketed plan's graph serves every batch of its
// bucket on this workspace and stream: the key is the parts' capacities;
// pixels, outputs, counts and descriptors are read on the device.  Otherwise the key is the exact batch and its pointers.
std::string graph_key(const Plan& p, const void* pix, const void* emb, const void* ws,
                      size_t ws_bytes, hipStream_t s) {
  std::string k;
  k.reserve(64 + 8 * p.n);
  auto put = [&](const void* v, size_t n) { k.append(static_cast<const char*>(v), n); };
  if (p.bucketed) {
    k.push_back('B');
    put(&ws, sizeof ws);
    put(&s, sizeof s);
    for (const Part& q : p.parts) {
      const int32_t c[2] = {q.T_cap, q.n_cap};
      put(c, sizeof c);
    }
    return k;
  }
  k.push_back('E');
  put(&pix, sizeof pix); put(&emb, sizeof emb); put(&ws, sizeof ws); put(&ws_bytes, sizeof ws_bytes);
  put(&s, sizeof s); put(&p.n, sizeof p.n);
  const size_t np = p.parts.size();
  put(&np, sizeof np);
  put(p.hw.data(), sizeof(int32_t) * p.hw.size());
  return k;
}

// Frees one cached graph once its last replay has finished.
void release_graph(GraphEntry& g) {
  if (g.done) {
    (void)hipEventSynchronize(g.done);
    (void)hipEventDestroy(g.done);
  }
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.host) (void)hipHostFree(g.host);
  g = GraphEntry{};
}

void destroy_graphs(vl_model* m) {
  for (auto& kv : m->graphs) release_graph(kv.second);
  m->graphs.clear();
}

// Drops the least recently replayed graph (waiting only for that graph).
void evict_graph(vl_model* m) {
  auto victim = m->graphs.end();
  for (auto it = m->graphs.begin(); it != m->graphs.end(); ++it)
    if (victim == m->graphs.end() || it->second.last_use < victim->second.last_use) victim = it;
  if (victim == m->graphs.end()) return;
  release_graph(victim->second);
  m->graphs.erase(victim);
}

// Records that the model's work so far on stream s ends here.
vl_status mark_use(vl_model* m, hipStream_t s) {
  hipEvent_t& ev = m->last_use[s];
  if (!ev) VL_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  VL_HIP(hipEventRecord(ev, s));
  return VL_OK;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

int32_t vl_abi_version(void) { return VL_ABI_VERSION; }

const char* vl_status_string(vl_status s) {
  switch (s) {
    case VL_OK: return "ok";
    case VL_ERR_INVALID_ARG: return "invalid argument";
    case VL_ERR_UNSUPPORTED: return "unsupported";
    case VL_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case VL_ERR_DEVICE: return "device error";
    case VL_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* vl_last_error_message(void) { return g_last_error.c_str(); }

size_t vl_weights_count(const vl_config* cfg) {
  std::string why;
  if (!config_ok(cfg, &why)) return 0;
  return weights_count(*cfg);
}

// Device copy of a model's weights in its precision (one hipMalloc), from the
// FP32 blob; m holds the dimensions.  Frees m on failure.
static vl_status build_weights(vl_model* m, const float* wdev, hipStream_t s, vl_model** out) {
  const vl_precision prec = m->prec;
  const size_t D = m->D, F = m->F;
  // position rows: image class token + g0 x g0 grid, or text context length
  const size_t G = m->text ? (size_t)m->ctx : 1 + (size_t)m->g0 * m->g0;

  // Source offsets in the FP32 blob (layout in include/vl.h).
  size_t o = 0;
  auto take = [&](size_t n) { size_t r = o; o += n; return wdev + r; };
  const float *s_patch_w = nullptr, *s_patch_b = nullptr, *s_cls = nullptr, *s_tok = nullptr;
  if (m->text) {
    s_tok = take((size_t)m->vocab * D);
  } else {
    s_patch_w = take(D * m->Kpe);
    s_patch_b = take(D);
    s_cls = take(D);
  }
  const float* s_pos = take(G * D);
  struct SrcLayer { const float *ln1_g, *ln1_b, *qkv_w, *qkv_b, *o_w, *o_b, *ln2_g, *ln2_b, *fc1_w, *fc1_b, *fc2_w, *fc2_b; };
  std::vector<SrcLayer> src(m->L);
  for (int l = 0; l < m->L; ++l) {
    SrcLayer& x = src[l];
    x.ln1_g = take(D); x.ln1_b = take(D); x.qkv_w = take(3 * D * D); x.qkv_b = take(3 * D);
    x.o_w = take(D * D); x.o_b = take(D); x.ln2_g = take(D); x.ln2_b = take(D);
    x.fc1_w = take(F * D); x.fc1_b = take(F); x.fc2_w = take(D * F); x.fc2_b = take(D);
  }
  const float* s_lnf_g = take(D);
  const float* s_lnf_b = take(D);
  const bool map = !m->text && m->cfg.pool == VL_POOL_MAP;
  struct SrcMap { const float *probe, *q_w, *q_b, *kv_w, *kv_b, *o_w, *o_b, *ln_g, *ln_b, *fc1_w, *fc1_b, *fc2_w, *fc2_b; } sm{};
  if (map) {
    sm.probe = take(D); sm.q_w = take(D * D); sm.q_b = take(D);
    sm.kv_w = take(2 * D * D); sm.kv_b = take(2 * D); sm.o_w = take(D * D); sm.o_b = take(D);
    sm.ln_g = take(D); sm.ln_b = take(D); sm.fc1_w = take(F * D); sm.fc1_b = take(F);
    sm.fc2_w = take(D * F); sm.fc2_b = take(D);
  }
  const float* s_proj = take((size_t)m->Pd * D);

  // Destination layout.
  const size_t wes = prec == VL_FP32 ? 4 : (prec == VL_BF16 ? 2 : 1);
  const size_t pes = prec == VL_FP32 ? 4 : 2;
  size_t sz = 0;
  auto alloc = [&](size_t bytes) { size_t r = sz; sz += align_up(bytes); return r; };
  const size_t d_patch_w = m->text ? 0 : alloc(pes * D * m->Kpad);
  const size_t d_patch_b = m->text ? 0 : alloc(4 * D);
  const size_t d_cls = m->text ? 0 : alloc(4 * D);
  const size_t d_tok = m->text ? alloc(4 * (size_t)m->vocab * D) : 0;
  const size_t d_pos = alloc(4 * G * D);
  struct DstLayer { size_t ln1_g, ln1_b, ln2_g, ln2_b, qkv_b, o_b, fc1_b, fc2_b, qkv_w, o_w, fc1_w, fc2_w, qkv_s, o_s, fc1_s, fc2_s, qkv_c1, qkv_c2, fc1_c1, fc1_c2; };
  const bool folds = prec == VL_BF16 || prec == VL_FP8W_BF16A;   // LayerNorm folding constants
  const bool mx = prec == VL_MXFP8;
  std::vector<DstLayer> dl(m->L);
  for (int l = 0; l < m->L; ++l) {
    DstLayer& x = dl[l];
    x.ln1_g = alloc(4 * D); x.ln1_b = alloc(4 * D); x.ln2_g = alloc(4 * D); x.ln2_b = alloc(4 * D);
    x.qkv_b = alloc(4 * 3 * D); x.o_b = alloc(4 * D); x.fc1_b = alloc(4 * F); x.fc2_b = alloc(4 * D);
    x.qkv_w = alloc(wes * 3 * D * D); x.o_w = alloc(wes * D * D);
    x.fc1_w = alloc(wes * F * D); x.fc2_w = alloc(wes * D * F);
    if (prec == VL_FP8W_BF16A) {
      x.qkv_s = alloc(4 * 3 * D); x.o_s = alloc(4 * D); x.fc1_s = alloc(4 * F); x.fc2_s = alloc(4 * D);
    }
    if (mx) {  // one E8M0 byte per 32 weights
      x.qkv_s = alloc(3 * D * D / 32); x.o_s = alloc(D * D / 32);
      x.fc1_s = alloc(F * D / 32); x.fc2_s = alloc(D * F / 32);
    }
    if (folds) {
      x.qkv_c1 = alloc(4 * 3 * D); x.qkv_c2 = alloc(4 * 3 * D);
      x.fc1_c1 = alloc(4 * F); x.fc1_c2 = alloc(4 * F);
    }
  }
  const size_t d_lnf_g = alloc(4 * D);
  const size_t d_lnf_b = alloc(4 * D);
  const size_t d_proj = alloc(4 * (size_t)m->Pd * D);
  struct DstMap { size_t q, kv_w, kv_b, o_w, o_b, ln_g, ln_b, fc1_w, fc1_b, fc2_w, fc2_b, probe, q_w; } dm{};
  if (map) {
    dm.q = alloc(4 * D); dm.probe = alloc(4 * D); dm.q_w = alloc(4 * D * D);
    dm.kv_w = alloc(pes * 2 * D * D); dm.kv_b = alloc(4 * 2 * D);
    dm.o_w = alloc(4 * D * D); dm.o_b = alloc(4 * D); dm.ln_g = alloc(4 * D); dm.ln_b = alloc(4 * D);
    dm.fc1_w = alloc(4 * F * D); dm.fc1_b = alloc(4 * F); dm.fc2_w = alloc(4 * D * F);
    dm.fc2_b = alloc(4 * D);
  }
  m->wbytes = sz;
  {
    hipError_t e = hipMalloc(&m->wmem, sz);
    if (e != hipSuccess) { delete m; return hip_fail(e, "hipMalloc(model weights)"); }
  }
  char* b = m->wmem;
  auto f = [&](size_t off) { return reinterpret_cast<float*>(b + off); };

  vl_status st = VL_OK;
  auto chk = [&](hipError_t e, const char* what) {
    if (st == VL_OK && e != hipSuccess) st = hip_fail(e, what);
  };
  if (m->text) {
    chk(copy_f32(s_tok, f(d_tok), (size_t)m->vocab * D, s), "copy token table");
  } else {
    chk(fold_patch_weights(s_patch_w, s_patch_b, m->cfg.chan_mean, m->cfg.chan_std,
                           m->cfg.channels, m->D, m->P, m->Kpad, prec == VL_FP32 ? f(d_patch_w) : nullptr,
                           prec == VL_FP32 ? nullptr : reinterpret_cast<bf16_t*>(b + d_patch_w),
                           f(d_patch_b), s),
        "fold_patch_weights");
    chk(copy_f32(s_cls, f(d_cls), D, s), "copy cls");
  }
  chk(copy_f32(s_pos, f(d_pos), G * D, s), "copy pos");
  auto conv_w = [&](const float* src_w, size_t dst_off, size_t scale_off, int rows, int cols) {
    if (prec == VL_FP32)
      chk(copy_f32(src_w, f(dst_off), (size_t)rows * cols, s), "copy weight");
    else if (prec == VL_BF16)
      chk(convert_bf16(src_w, reinterpret_cast<bf16_t*>(b + dst_off), (size_t)rows * cols, s),
          "convert_bf16");
    else if (prec == VL_MXFP8)
      chk(mx_quantise_rows(src_w, reinterpret_cast<uint8_t*>(b + dst_off),
                           reinterpret_cast<uint8_t*>(b + scale_off), rows, cols, s),
          "mx_quantise_rows");
    else
      chk(quantise_e4m3_rows(src_w, reinterpret_cast<uint8_t*>(b + dst_off), f(scale_off), rows,
                             cols, s),
          "quantise_e4m3_rows");
  };
  m->layers.resize(m->L);
  for (int l = 0; l < m->L; ++l) {
    const SrcLayer& x = src[l];
    const DstLayer& y = dl[l];
    chk(copy_f32(x.ln1_g, f(y.ln1_g), D, s), "copy");
    chk(copy_f32(x.ln1_b, f(y.ln1_b), D, s), "copy");
    chk(copy_f32(x.ln2_g, f(y.ln2_g), D, s), "copy");
    chk(copy_f32(x.ln2_b, f(y.ln2_b), D, s), "copy");
    chk(copy_f32(x.qkv_b, f(y.qkv_b), 3 * D, s), "copy");
    chk(copy_f32(x.o_b, f(y.o_b), D, s), "copy");
    chk(copy_f32(x.fc1_b, f(y.fc1_b), F, s), "copy");
    chk(copy_f32(x.fc2_b, f(y.fc2_b), D, s), "copy");
    conv_w(x.qkv_w, y.qkv_w, y.qkv_s, 3 * m->D, m->D);
    conv_w(x.o_w, y.o_w, y.o_s, m->D, m->D);
    conv_w(x.fc1_w, y.fc1_w, y.fc1_s, m->F, m->D);
    conv_w(x.fc2_w, y.fc2_w, y.fc2_s, m->D, m->F);
    Layer& ly = m->layers[l];
    ly.ln1_g = f(y.ln1_g); ly.ln1_b = f(y.ln1_b); ly.ln2_g = f(y.ln2_g); ly.ln2_b = f(y.ln2_b);
    ly.qkv_b = f(y.qkv_b); ly.o_b = f(y.o_b); ly.fc1_b = f(y.fc1_b); ly.fc2_b = f(y.fc2_b);
    ly.qkv_w = b + y.qkv_w; ly.o_w = b + y.o_w; ly.fc1_w = b + y.fc1_w; ly.fc2_w = b + y.fc2_w;
    const bool q8 = prec == VL_FP8W_BF16A;
    ly.qkv_s = q8 ? f(y.qkv_s) : nullptr; ly.o_s = q8 ? f(y.o_s) : nullptr;
    ly.fc1_s = q8 ? f(y.fc1_s) : nullptr; ly.fc2_s = q8 ? f(y.fc2_s) : nullptr;
    auto u8 = [&](size_t off) { return mx ? reinterpret_cast<const uint8_t*>(b + off) : nullptr; };
    ly.qkv_x = u8(y.qkv_s); ly.o_x = u8(y.o_s); ly.fc1_x = u8(y.fc1_s); ly.fc2_x = u8(y.fc2_s);
    if (folds) {
      // from the converted weights (stream order: after their conversion)
      chk(ln_fold_consts(ly.qkv_w, q8, ly.qkv_s, ly.ln1_g, ly.ln1_b, ly.qkv_b, 3 * m->D, m->D,
                         f(y.qkv_c1), f(y.qkv_c2), s),
          "ln_fold_consts");
      chk(ln_fold_consts(ly.fc1_w, q8, ly.fc1_s, ly.ln2_g, ly.ln2_b, ly.fc1_b, m->F, m->D,
                         f(y.fc1_c1), f(y.fc1_c2), s),
          "ln_fold_consts");
      ly.qkv_c1 = f(y.qkv_c1); ly.qkv_c2 = f(y.qkv_c2);
      ly.fc1_c1 = f(y.fc1_c1); ly.fc1_c2 = f(y.fc1_c2);
    }
  }
  chk(copy_f32(s_lnf_g, f(d_lnf_g), D, s), "copy");
  chk(copy_f32(s_lnf_b, f(d_lnf_b), D, s), "copy");
  chk(copy_f32(s_proj, f(d_proj), (size_t)m->Pd * D, s), "copy");
  if (map) {
    // q = probe W_q^T + b_q once (FP32 GEMM, one row)
    EpiArgs eq;
    eq.bias = sm.q_b;
    eq.out = f(dm.q);
    eq.ldo = (int)D;
    chk(gemm_f32(sm.probe, (int)D, sm.q_w, (int)D, 1, (int)D, (int)D, OP_QKV, eq, s), "map query");
    chk(copy_f32(sm.probe, f(dm.probe), D, s), "copy");
    chk(copy_f32(sm.q_w, f(dm.q_w), D * D, s), "copy");
    if (prec == VL_FP32)
      chk(copy_f32(sm.kv_w, f(dm.kv_w), 2 * D * D, s), "copy");
    else
      chk(convert_bf16(sm.kv_w, reinterpret_cast<bf16_t*>(b + dm.kv_w), 2 * D * D, s), "convert_bf16");
    chk(copy_f32(sm.kv_b, f(dm.kv_b), 2 * D, s), "copy");
    chk(copy_f32(sm.o_w, f(dm.o_w), D * D, s), "copy");
    chk(copy_f32(sm.o_b, f(dm.o_b), D, s), "copy");
    chk(copy_f32(sm.ln_g, f(dm.ln_g), D, s), "copy");
    chk(copy_f32(sm.ln_b, f(dm.ln_b), D, s), "copy");
    chk(copy_f32(sm.fc1_w, f(dm.fc1_w), F * D, s), "copy");
    chk(copy_f32(sm.fc1_b, f(dm.fc1_b), F, s), "copy");
    chk(copy_f32(sm.fc2_w, f(dm.fc2_w), D * F, s), "copy");
    chk(copy_f32(sm.fc2_b, f(dm.fc2_b), D, s), "copy");
    m->map_q = f(dm.q); m->map_kv_w = b + dm.kv_w; m->map_kv_b = f(dm.kv_b);
    m->map_o_w = f(dm.o_w); m->map_o_b = f(dm.o_b); m->map_ln_g = f(dm.ln_g); m->map_ln_b = f(dm.ln_b);
    m->map_fc1_w = f(dm.fc1_w); m->map_fc1_b = f(dm.fc1_b); m->map_fc2_w = f(dm.fc2_w);
    m->map_fc2_b = f(dm.fc2_b);
    m->map_probe = f(dm.probe); m->map_q_w = f(dm.q_w);
  }
  if (m->text) {
    m->tok_emb = f(d_tok);
  } else {
    m->patch_w = b + d_patch_w;
    m->patch_b = f(d_patch_b);
    m->cls = f(d_cls);
  }
  m->pos = f(d_pos);
  m->lnf_g = f(d_lnf_g);
  m->lnf_b = f(d_lnf_b);
  m->proj = f(d_proj);
  for (auto& row : m->tuning)
    for (auto& v : row) v = -1;
  m->ring.resize(8);
  for (Staging& r : m->ring) chk(hipEventCreateWithFlags(&r.ev, hipEventDisableTiming), "hipEventCreate");
  if (st == VL_OK) st = mark_use(m, s);   // destroy waits for the conversion kernels
  if (st != VL_OK) {
    vl_model_destroy(m);
    return st;
  }
  *out = m;
  return VL_OK;
}

size_t vl_text_weights_count(const vl_text_config* cfg) {
  std::string why;
  if (!text_config_ok(cfg, &why)) return 0;
  return text_weights_count(*cfg);
}

vl_status vl_text_model_create(const vl_text_config* cfg, vl_precision prec, const float* wdev,
                               size_t n_floats, void* stream, vl_model** out) {
  std::string why;
  if (!out) return fail(VL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!text_config_ok(cfg, &why)) return fail(VL_ERR_INVALID_ARG, why);
  if (!wdev) return fail(VL_ERR_INVALID_ARG, "weights_dev is NULL");
  if (prec != VL_FP32 && prec != VL_BF16 && prec != VL_FP8W_BF16A && prec != VL_MXFP8)
    return fail(VL_ERR_INVALID_ARG, "unknown precision");
  if (n_floats != text_weights_count(*cfg))
    return fail(VL_ERR_INVALID_ARG, "weight blob has " + std::to_string(n_floats) +
                                        " floats, expected " +
                                        std::to_string(text_weights_count(*cfg)));
  const int hd = cfg->width / cfg->heads;
  if (hd != 32 && hd != 64) return fail(VL_ERR_UNSUPPORTED, "head_dim must be 32 or 64");
  if (cfg->width > 1024) return fail(VL_ERR_UNSUPPORTED, "width must be <= 1024");
  vl_model* m = new vl_model();
  m->text = true;
  m->prec = prec;
  if (hipGetDevice(&m->device) != hipSuccess) { delete m; return fail(VL_ERR_DEVICE, "hipGetDevice failed"); }
  m->cfg = vl_config{};
  m->cfg.ln_eps = cfg->ln_eps;
  m->vocab = cfg->vocab; m->ctx = cfg->ctx;
  m->D = cfg->width; m->F = cfg->mlp; m->heads = cfg->heads; m->hd = hd; m->L = cfg->layers;
  m->Pd = cfg->proj_dim;
  m->P = 0; m->g0 = 0; m->Kpe = 0; m->Kpad = 0;
  return build_weights(m, wdev, static_cast<hipStream_t>(stream), out);
}

vl_status vl_model_create(const vl_config* cfg, vl_precision prec, const float* wdev,
                          size_t n_floats, void* stream, vl_model** out) {
  std::string why;
  if (!out) return fail(VL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!config_ok(cfg, &why)) return fail(VL_ERR_INVALID_ARG, why);
  if (!wdev) return fail(VL_ERR_INVALID_ARG, "weights_dev is NULL");
  if (prec != VL_FP32 && prec != VL_BF16 && prec != VL_FP8W_BF16A && prec != VL_MXFP8)
    return fail(VL_ERR_INVALID_ARG, "unknown precision");
  if (n_floats != weights_count(*cfg))
    return fail(VL_ERR_INVALID_ARG, "weight blob has " + std::to_string(n_floats) +
                                        " floats, expected " + std::to_string(weights_count(*cfg)));
  const int hd = cfg->width / cfg->heads;
  if (hd != 32 && hd != 64) return fail(VL_ERR_UNSUPPORTED, "head_dim must be 32 or 64");
  if (cfg->width > 1024) return fail(VL_ERR_UNSUPPORTED, "width must be <= 1024");

  vl_model* m = new vl_model();
  m->cfg = *cfg;
  m->prec = prec;
  if (hipGetDevice(&m->device) != hipSuccess) { delete m; return fail(VL_ERR_DEVICE, "hipGetDevice failed"); }
  m->D = cfg->width; m->F = cfg->mlp; m->heads = cfg->heads; m->hd = hd; m->L = cfg->layers;
  m->P = cfg->patch; m->Pd = cfg->proj_dim; m->g0 = cfg->base_grid;
  m->Kpe = cfg->channels * m->P * m->P;
  m->Kpad = (m->Kpe + 63) / 64 * 64;
  return build_weights(m, wdev, static_cast<hipStream_t>(stream), out);
}

void vl_model_destroy(vl_model* m) {
  if (!m) return;
  // Wait for the model's own enqueued work: every stream it was used on,
  // its side stream, pending descriptor copies and cached graphs.
  for (auto& kv : m->last_use) {
    (void)hipEventSynchronize(kv.second);
    (void)hipEventDestroy(kv.second);
  }
  m->last_use.clear();
  if (m->side) (void)hipStreamSynchronize(m->side);
  for (Staging& r : m->ring)
    if (r.pending && r.ev) (void)hipEventSynchronize(r.ev);
  destroy_graphs(m);
  for (TimedLaunch& t : m->timed) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (hipEvent_t e : m->free_events) (void)hipEventDestroy(e);
  for (Staging& r : m->ring) {
    if (r.host) (void)hipHostFree(r.host);
    if (r.ev) (void)hipEventDestroy(r.ev);
  }
  if (m->capture) (void)hipStreamDestroy(m->capture);
  if (m->side) (void)hipStreamDestroy(m->side);
  if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
  if (m->ev_join) (void)hipEventDestroy(m->ev_join);
  for (hipEvent_t e : m->tev)
    if (e) (void)hipEventDestroy(e);
  if (m->wmem) (void)hipFree(m->wmem);
  if (m->wT) (void)hipFree(m->wT);
  if (m->wT_ev) (void)hipEventDestroy(m->wT_ev);
  delete m;
}

vl_status vl_model_set_option(vl_model* m, vl_option opt, int64_t value) {
  if (!m) return fail(VL_ERR_INVALID_ARG, "model is NULL");
  std::lock_guard<std::mutex> lk(m->mu);
  switch (opt) {
    case VL_OPT_GRAPHS:
      m->use_graphs = value != 0;
      if (!m->use_graphs) destroy_graphs(m);
      return VL_OK;
    case VL_OPT_TIMING:
      m->timing = value != 0;
      return VL_OK;
    case VL_OPT_SPLIT:
      destroy_graphs(m);
      m->split = value != 0;
      return VL_OK;
    case VL_OPT_FUSED_LN:
      destroy_graphs(m);
      m->fused_ln = value != 0;
      return VL_OK;
    case VL_OPT_ATTN_RESIDENT:
      destroy_graphs(m);
      m->attn_resident = value != 0;
      return VL_OK;
    case VL_OPT_GRAPH_BUCKETS:
      destroy_graphs(m);
      m->graph_buckets = value != 0;
      return VL_OK;
    case VL_OPT_KMAJOR_WGRAD:
      m->kmajor_wgrad = value != 0;
      return VL_OK;
  }
  return fail(VL_ERR_INVALID_ARG, "unknown option");
}

vl_status vl_model_op_times(vl_model* m, double* ms_out, int64_t* launches_out, int32_t reset) {
  if (!m) return fail(VL_ERR_INVALID_ARG, "model is NULL");
  std::lock_guard<std::mutex> lk(m->mu);
  for (TimedLaunch& t : m->timed) {
    VL_HIP(hipEventSynchronize(t.stop));
    float ms = 0.f;
    VL_HIP(hipEventElapsedTime(&ms, t.start, t.stop));
    m->op_ms[t.op] += ms;
    m->op_launches[t.op] += 1;
    m->free_events.push_back(t.start);
    m->free_events.push_back(t.stop);
  }
  m->timed.clear();
  for (int i = 0; i < VL_N_OPS; ++i) {
    if (ms_out) ms_out[i] = m->op_ms[i];
    if (launches_out) launches_out[i] = m->op_launches[i];
    if (reset) {
      m->op_ms[i] = 0.0;
      m->op_launches[i] = 0;
    }
  }
  return VL_OK;
}

vl_status vl_model_graph_stats(vl_model* m, int64_t* captures, int64_t* replays,
                               int32_t* cached) {
  if (!m) return fail(VL_ERR_INVALID_ARG, "model is NULL");
  std::lock_guard<std::mutex> lk(m->mu);
  if (captures) *captures = m->graph_captures;
  if (replays) *replays = m->graph_replays;
  if (cached) *cached = (int32_t)m->graphs.size();
  return VL_OK;
}

size_t vl_encode_workspace_bytes(const vl_model* m, int32_t n, const int32_t* hs,
                                 const int32_t* ws) {
  if (!m) return 0;
  Plan p;
  std::string why;
  if (!make_plan(m, n, hs, ws, &p, &why, false, bucket_mode(m))) return 0;
  return p.total;
}

// Enqueue (or capture and replay) the kernel sequence of a planned batch.
static vl_status encode_planned(vl_model* m, const Plan& p, const void* pix, float* emb, void* ws,
                                size_t ws_bytes, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  std::lock_guard<std::mutex> lk(m->mu);
  if (!m->use_graphs || m->timing) {
    vl_status st = stage_descriptors(m, p, w, s);
    if (st == VL_OK) st = run_encoder(m, p, pix, emb, w, s);
    if (st != VL_OK) return st;
    return mark_use(m, s);
  }
  // A bucketed graph reads this call's descriptors, uploaded ahead of it on
  // the same stream; an exact-key graph holds its own upload.
  if (p.bucketed) {
    const vl_status st0 = stage_descriptors(m, p, w, s);
    if (st0 != VL_OK) return st0;
  }
  const std::string key = graph_key(p, pix, emb, ws, ws_bytes, s);
  auto it = m->graphs.find(key);
  if (it == m->graphs.end()) {
    while (m->graphs.size() >= kMaxGraphs) evict_graph(m);
    // Capture on the model's private stream (the caller's stream may be the
    // null stream, which cannot be captured); the graph is replayed on the
    // caller's stream.  Capture records work without running it.
    if (!m->capture) VL_HIP(hipStreamCreateWithFlags(&m->capture, hipStreamNonBlocking));
    hipStream_t cs = m->capture;
    GraphEntry ge;
    if (!p.bucketed) {
      VL_HIP(hipHostMalloc(&ge.host, std::max<size_t>(p.desc_bytes, 256), hipHostMallocDefault));
      std::memcpy(ge.host, p.desc.data(), p.desc_bytes);
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      if (ge.host) (void)hipHostFree(ge.host);
      return hip_fail(e, "hipStreamBeginCapture");
    }
    vl_status st = VL_OK;
    if (!p.bucketed) {
      e = hipMemcpyAsync(w, ge.host, p.desc_bytes, hipMemcpyHostToDevice, cs);
      if (e != hipSuccess) st = hip_fail(e, "hipMemcpyAsync(descriptors)");
    }
    if (st == VL_OK) st = run_encoder(m, p, pix, emb, w, cs);
    e = hipStreamEndCapture(cs, &g);
    if (st == VL_OK && e != hipSuccess) st = hip_fail(e, "hipStreamEndCapture");
    if (st == VL_OK) {
      e = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
      if (e != hipSuccess) st = hip_fail(e, "hipGraphInstantiate");
    }
    if (g) (void)hipGraphDestroy(g);
    if (st == VL_OK) {
      e = hipEventCreateWithFlags(&ge.done, hipEventDisableTiming);
      if (e != hipSuccess) st = hip_fail(e, "hipEventCreate");
    }
    if (st != VL_OK) { release_graph(ge); return st; }
    it = m->graphs.emplace(key, ge).first;
    ++m->graph_captures;
  }
  VL_HIP(hipGraphLaunch(it->second.exec, s));
  VL_HIP(hipEventRecord(it->second.done, s));
  it->second.last_use = ++m->graph_clock;
  ++m->graph_replays;
  return mark_use(m, s);
}

vl_status vl_encode_images(vl_model* m, const float* pix, const int32_t* hs, const int32_t* wsz,
                           int32_t n, float* emb, void* ws, size_t ws_bytes, void* stream) {
  if (!m) return fail(VL_ERR_INVALID_ARG, "model is NULL");
  if (!pix || !emb || !ws) return fail(VL_ERR_INVALID_ARG, "pixels, emb_out or workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(VL_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (reinterpret_cast<uintptr_t>(pix) % 16 || reinterpret_cast<uintptr_t>(emb) % 16)
    return fail(VL_ERR_INVALID_ARG, "pixels and emb_out must be 16-byte aligned");
  Plan p;
  std::string why;
  if (!make_plan(m, n, hs, wsz, &p, &why, false, bucket_mode(m)))
    return fail(VL_ERR_INVALID_ARG, why);
  if (ws_bytes < p.total)
    return fail(VL_ERR_WORKSPACE_TOO_SMALL, "workspace has " + std::to_string(ws_bytes) +
                                                " bytes, needs " + std::to_string(p.total));
  bind_batch(p, pix, emb, m->Pd);
  return encode_planned(m, p, pix, emb, ws, ws_bytes, stream);
}

size_t vl_text_workspace_bytes(const vl_model* m, int32_t n, const int32_t* lens) {
  if (!m) return 0;
  Plan p;
  std::string why;
  if (!make_text_plan(m, n, lens, &p, &why)) return 0;
  return p.total;
}

vl_status vl_encode_texts(vl_model* m, const int32_t* ids, const int32_t* lens, int32_t n,
                          float* emb, void* ws, size_t ws_bytes, void* stream) {
  if (!m) return fail(VL_ERR_INVALID_ARG, "model is NULL");
  if (!ids || !emb || !ws) return fail(VL_ERR_INVALID_ARG, "ids, emb_out or workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(VL_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (reinterpret_cast<uintptr_t>(ids) % 4 || reinterpret_cast<uintptr_t>(emb) % 16)
    return fail(VL_ERR_INVALID_ARG, "ids must be 4-byte and emb_out 16-byte aligned");
  Plan p;
  std::string why;
  if (!make_text_plan(m, n, lens, &p, &why)) return fail(VL_ERR_INVALID_ARG, why);
  if (ws_bytes < p.total)
    return fail(VL_ERR_WORKSPACE_TOO_SMALL, "workspace has " + std::to_string(ws_bytes) +
                                                " bytes, needs " + std::to_string(p.total));
  return encode_planned(m, p, ids, emb, ws, ws_bytes, stream);
}

int32_t vl_gemm_config_count(void) { return N_GEMM_CFGS; }

const char* vl_gemm_config_name(int32_t cfg) {
  return cfg >= 0 && cfg < N_GEMM_CFGS ? gemm_cfg_name(cfg) : nullptr;
}

vl_status vl_model_get_tuning(const vl_model* m, int32_t* table) {
  if (!m || !table) return fail(VL_ERR_INVALID_ARG, "NULL argument");
  std::memcpy(table, m->tuning, sizeof(m->tuning));
  return VL_OK;
}

vl_status vl_model_set_tuning(vl_model* m, const int32_t* table) {
  if (!m || !table) return fail(VL_ERR_INVALID_ARG, "NULL argument");
  for (int i = 0; i < VL_N_GEMM_OPS * VL_N_M_BUCKETS; ++i)
    if (table[i] < -1 || table[i] >= N_GEMM_CFGS)
      return fail(VL_ERR_INVALID_ARG, "tuning entry " + std::to_string(i) + " is not a configuration id");
  std::lock_guard<std::mutex> lk(m->mu);
  destroy_graphs(m);
  std::memcpy(m->tuning, table, sizeof(m->tuning));
  return VL_OK;
}

vl_status vl_model_autotune(vl_model* m, const float* pix, const int32_t* hs, const int32_t* wsz,
                            int32_t n, float* emb, void* ws, size_t ws_bytes, int32_t reps,
                            void* stream) {
  if (!m) return fail(VL_ERR_INVALID_ARG, "model is NULL");
  if (m->prec == VL_FP32) return fail(VL_ERR_UNSUPPORTED, "FP32 models have a single GEMM");
  if (reps < 1) return fail(VL_ERR_INVALID_ARG, "reps must be >= 1");
  if (!pix || !emb || !ws) return fail(VL_ERR_INVALID_ARG, "pixels, emb_out or workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(VL_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  Plan p;
  std::string why;
  if (!make_plan(m, n, hs, wsz, &p, &why)) return fail(VL_ERR_INVALID_ARG, why);
  if (ws_bytes < p.total) return fail(VL_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  std::lock_guard<std::mutex> lk(m->mu);
  const bool timing = m->timing;
  m->timing = false;
  vl_status st = stage_descriptors(m, p, w, s);
  if (st == VL_OK) st = run_encoder(m, p, pix, emb, w, s);
  m->timing = timing;
  if (st != VL_OK) return st;
  const bool fp8 = m->prec == VL_FP8W_BF16A;
  const int D = m->D, F = m->F;
  const Layer& ly = m->layers.empty() ? Layer{} : m->layers[0];
  hipEvent_t e0, e1;
  VL_HIP(hipEventCreate(&e0));
  VL_HIP(hipEventCreate(&e1));
  // Tune each distinct part size (M bucket) on that part's buffers, which
  // the run above filled with this batch's activations.
  bool tuned[VL_N_M_BUCKETS] = {};
  // Kernel-level times of every configuration per operation (last bucket).
  std::vector<std::pair<float, int>> cand[VL_N_GEMM_OPS];
  for (const Part& q : p.parts) {
    const int T = q.T;
    const int b = m_bucket(T);
    if (tuned[b]) continue;
    tuned[b] = true;
    const bf16_t* Y = reinterpret_cast<const bf16_t*>(w + q.off_Y);
    bf16_t* QH = reinterpret_cast<bf16_t*>(w + q.off_QH);
    float* X = reinterpret_cast<float*>(w + q.off_X);
    const int2* tok = reinterpret_cast<const int2*>(w + q.off_tok);
    struct OpShape {
      int op, N, K; const bf16_t* A; int lda; const void* B; bool b8; EpiArgs e;
      const uint8_t *a8 = nullptr, *sa = nullptr, *sb = nullptr;  // MXFP8 operands
    };
    std::vector<OpShape> shapes;
    {
      EpiArgs pe;
      pe.bias = m->patch_b; pe.out = X; pe.ldo = D; pe.tok_info = tok;
      pe.imgs = reinterpret_cast<const ImgDesc*>(w + q.off_imgs); pe.cls = m->cls; pe.pos = m->pos;
      pe.base_grid = m->g0;
      shapes.push_back({OP_PATCH, D, m->Kpad, QH, m->Kpad, m->patch_w, false, pe});
    }
    if (!m->layers.empty()) {
      EpiArgs e1a; e1a.bias = ly.qkv_b; e1a.wscale = ly.qkv_s; e1a.out = QH; e1a.ldo = 3 * D;
      EpiArgs e2a; e2a.bias = ly.o_b; e2a.wscale = ly.o_s; e2a.out = X; e2a.ldo = D;
      EpiArgs e3a; e3a.bias = ly.fc1_b; e3a.wscale = ly.fc1_s; e3a.out = QH; e3a.ldo = F;
      EpiArgs e4a; e4a.bias = ly.fc2_b; e4a.wscale = ly.fc2_s; e4a.out = X; e4a.ldo = D;
      const bf16_t* a_ln = Y;
      if (m->fused_ln && m->prec != VL_MXFP8) {   // time the folded epilogues
        bf16_t* U = reinterpret_cast<bf16_t*>(w + q.off_U);
        float* RS = reinterpret_cast<float*>(w + q.off_RS);
        a_ln = U;
        e1a.row_stats = RS; e1a.c1 = ly.qkv_c1; e1a.c2 = ly.qkv_c2;
        e3a.row_stats = RS; e3a.c1 = ly.fc1_c1; e3a.c2 = ly.fc1_c2;
        e2a.u_out = U; e2a.u_gamma = ly.ln2_g;
        e2a.part_stats = reinterpret_cast<float*>(w + q.off_PS);
        e4a.u_out = U; e4a.u_gamma = ly.ln1_g; e4a.part_stats = e2a.part_stats;
      }
      shapes.push_back({OP_QKV, 3 * D, D, a_ln, D, ly.qkv_w, fp8, e1a});
      shapes.push_back({OP_OPROJ, D, D, Y, D, ly.o_w, fp8, e2a});
      shapes.push_back({OP_FC1, F, D, a_ln, D, ly.fc1_w, fp8, e3a});
      shapes.push_back({OP_FC2, D, F, QH, F, ly.fc2_w, fp8, e4a});
      if (m->prec == VL_MXFP8) {
        const uint8_t* y8 = reinterpret_cast<const uint8_t*>(Y);
        const uint8_t* h8 = reinterpret_cast<const uint8_t*>(QH);
        const uint8_t* sx[4] = {ly.qkv_x, ly.o_x, ly.fc1_x, ly.fc2_x};
        for (int i = 1; i <= 4; ++i) {
          OpShape& o = shapes[i];
          o.a8 = o.op == OP_FC2 ? h8 : y8;
          o.sa = o.a8 + (size_t)T * o.K;
          o.sb = sx[i - 1];
        }
        shapes[3].e.out = QH;
        shapes[3].e.out_scale = reinterpret_cast<uint8_t*>(QH) + (size_t)T * F;
        shapes[3].e.scale_rows = T;
      }
    }
    for (const OpShape& o : shapes) {
      float best = 1e30f;
      int best_cfg = -1;
      cand[o.op].clear();
      const bool omx = o.a8 != nullptr;
      auto launch = [&](int cfg) {
        return omx ? gemm_mx(o.a8, o.sa, static_cast<const uint8_t*>(o.B), o.sb, T, o.N, o.K,
                             o.op, cfg, o.e, s)
                   : gemm_bf16(o.A, o.lda, o.B, o.K, o.b8, T, o.N, o.K, o.op, cfg, o.e, s);
      };
      for (int cfg = omx ? N_BF16_CFGS : 0; cfg < (omx ? N_GEMM_CFGS : N_BF16_CFGS); ++cfg) {
        hipError_t err = launch(cfg);
        if (err != hipSuccess) continue;
        VL_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) VL_HIP(launch(cfg));
        VL_HIP(hipEventRecord(e1, s));
        VL_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        VL_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) { best = ms; best_cfg = cfg; }
        cand[o.op].push_back({ms, cfg});
      }
      m->tuning[o.op][b] = best_cfg;
    }
  }
  // Kernel-level timing repeats one launch on warm operands; in the model
  // each layer's weights come from HBM and the A operand was just written,
  // which can reorder configurations a few per cent apart.  When the batch
  // runs as parts of one M bucket, the final choice per operation among the
  // configurations within 5 % of its fastest comes from timing whole
  // encoder passes (operations in turn, the others at their current pick).
  bool one_bucket = true;
  for (const Part& q : p.parts) one_bucket &= m_bucket(q.T) == m_bucket(p.parts[0].T);
  if (one_bucket && !m->layers.empty()) {
    const int b = m_bucket(p.parts[0].T);
    m->timing = false;
    for (int op = OP_QKV; op <= OP_FC2 && st == VL_OK; ++op) {
      std::vector<std::pair<float, int>>& c = cand[op];
      std::sort(c.begin(), c.end());
      int nc = 0;
      while (nc < (int)c.size() && nc < 3 && c[nc].first <= 1.05f * c[0].first) ++nc;
      if (nc < 2) continue;
      float best = 1e30f;
      int best_cfg = m->tuning[op][b];
      for (int i = 0; i < nc && st == VL_OK; ++i) {
        m->tuning[op][b] = c[i].second;
        st = run_encoder(m, p, pix, emb, w, s);   // warm-up with this choice
        if (st != VL_OK) break;
        VL_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps && st == VL_OK; ++r) st = run_encoder(m, p, pix, emb, w, s);
        VL_HIP(hipEventRecord(e1, s));
        VL_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        VL_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) { best = ms; best_cfg = c[i].second; }
      }
      m->tuning[op][b] = best_cfg;
    }
    m->timing = timing;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == VL_OK) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
  }
  destroy_graphs(m);
  return st;
}

vl_status vl_mx_quantize(const float* src, int32_t rows, int32_t cols, uint8_t* codes,
                         uint8_t* scales, void* stream) {
  if (!src || !codes || !scales) return fail(VL_ERR_INVALID_ARG, "NULL pointer argument");
  if (rows <= 0 || cols <= 0) return fail(VL_ERR_INVALID_ARG, "sizes must be > 0");
  if (cols % 128) return fail(VL_ERR_INVALID_ARG, "cols must be a multiple of 128");
  if (reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(codes) % 4)
    return fail(VL_ERR_INVALID_ARG, "src must be 16-byte and codes 4-byte aligned");
  VL_HIP(mx_quantise_rows(src, codes, scales, rows, cols, static_cast<hipStream_t>(stream)));
  return VL_OK;
}

vl_status vl_mx_gemm(const uint8_t* a, const uint8_t* sa, const uint8_t* b, const uint8_t* sb,
                     int32_t M, int32_t N, int32_t K, const float* bias, float* c, int32_t cfg,
                     void* stream) {
  if (!a || !sa || !b || !sb || !bias || !c) return fail(VL_ERR_INVALID_ARG, "NULL pointer argument");
  if (M <= 0 || N <= 0 || K <= 0) return fail(VL_ERR_INVALID_ARG, "sizes must be > 0");
  if (K % 128 || N % 32) return fail(VL_ERR_INVALID_ARG, "K must be a multiple of 128 and N of 32");
  if ((uint64_t)(K / 128) * ((uint64_t)std::max(M, N) + 256) * 4 >= (1ull << 32))
    return fail(VL_ERR_INVALID_ARG, "scale arrays exceed 4 GiB");
  if (cfg != -1 && !gemm_cfg_is_mx(cfg)) return fail(VL_ERR_INVALID_ARG, "cfg is not an MXFP8 configuration");
  auto al = [](const void* p, uintptr_t n) { return reinterpret_cast<uintptr_t>(p) % n == 0; };
  if (!al(a, 16) || !al(b, 16) || !al(c, 16) || !al(bias, 16) || !al(sa, 4) || !al(sb, 4))
    return fail(VL_ERR_INVALID_ARG, "codes, c and bias must be 16-byte, scales 4-byte aligned");
  EpiArgs e;
  e.bias = bias;
  e.out = c;
  e.ldo = N;
  VL_HIP(gemm_mx(a, sa, b, sb, M, N, K, OP_OPROJ, cfg, e, static_cast<hipStream_t>(stream)));
  return VL_OK;
}

size_t vl_contrastive_workspace_bytes(int32_t n, int32_t dim) {
  if (n <= 0 || dim <= 0) return 0;
  return contrastive_workspace_bytes(n, dim);
}

vl_status vl_contrastive_loss(const float* emb, const float* texts, int32_t n, int32_t dim,
                              vl_head head, float scale, float bias, float* loss, float* d_emb,
                              float* d_texts, float* d_scale_bias, void* ws, size_t ws_bytes,
                              void* stream) {
  if (!emb || !texts || !loss || !d_emb || !d_texts || !d_scale_bias || !ws)
    return fail(VL_ERR_INVALID_ARG, "NULL pointer argument");
  if (n <= 0 || dim <= 0) return fail(VL_ERR_INVALID_ARG, "sizes must be > 0");
  if (n > 65535) return fail(VL_ERR_INVALID_ARG, "n must be <= 65535");
  if (dim % 16) return fail(VL_ERR_INVALID_ARG, "dim must be a multiple of 16");
  if (head != VL_HEAD_SOFTMAX && head != VL_HEAD_SIGMOID) return fail(VL_ERR_INVALID_ARG, "unknown head");
  if (!std::isfinite(scale) || !(scale > 0.f) || !std::isfinite(bias))
    return fail(VL_ERR_INVALID_ARG, "scale must be finite and > 0, bias finite");
  auto al = [](const void* p, uintptr_t k) { return reinterpret_cast<uintptr_t>(p) % k == 0; };
  if (!al(emb, 16) || !al(texts, 16) || !al(d_emb, 16) || !al(d_texts, 16) || !al(ws, kAlign))
    return fail(VL_ERR_INVALID_ARG, "arrays must be 16-byte and the workspace 256-byte aligned");
  if (ws_bytes < contrastive_workspace_bytes(n, dim))
    return fail(VL_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
  VL_HIP(contrastive_loss(emb, texts, n, dim, head == VL_HEAD_SOFTMAX ? 0 : 1, scale, bias, loss,
                          d_emb, d_texts, d_scale_bias, ws, static_cast<hipStream_t>(stream)));
  return VL_OK;
}

vl_status vl_contrastive_loss_noalloc(const float* emb, const float* texts, int32_t n,
                                      int32_t dim, vl_head head, float scale, float bias,
                                      float* loss, float* d_emb, float* d_texts,
                                      float* d_scale_bias, void* stream) {
  if (!emb || !texts || !loss || !d_emb || !d_texts || !d_scale_bias)
    return fail(VL_ERR_INVALID_ARG, "NULL pointer argument");
  if (n <= 0 || dim <= 0) return fail(VL_ERR_INVALID_ARG, "sizes must be > 0");
  if (n > 65535) return fail(VL_ERR_INVALID_ARG, "n must be <= 65535");
  if (dim % 16) return fail(VL_ERR_INVALID_ARG, "dim must be a multiple of 16");
  if (head != VL_HEAD_SOFTMAX && head != VL_HEAD_SIGMOID) return fail(VL_ERR_INVALID_ARG, "unknown head");
  if (!std::isfinite(scale) || !(scale > 0.f) || !std::isfinite(bias))
    return fail(VL_ERR_INVALID_ARG, "scale must be finite and > 0, bias finite");
  auto al = [](const void* p, uintptr_t k) { return reinterpret_cast<uintptr_t>(p) % k == 0; };
  if (!al(emb, 16) || !al(texts, 16) || !al(d_emb, 16) || !al(d_texts, 16))
    return fail(VL_ERR_INVALID_ARG, "arrays must be 16-byte aligned");
  const size_t need = contrastive_workspace_bytes(n, dim);
  if (need > kNoAllocScratchBytes)
    return fail(VL_ERR_WORKSPACE_TOO_SMALL,
                "n = " + std::to_string(n) + ", dim = " + std::to_string(dim) + " needs " +
                    std::to_string(need) + " bytes of scratch; the allocation-free entry point "
                    "has " + std::to_string(kNoAllocScratchBytes) +
                    " (use vl_contrastive_loss with a caller workspace)");
  void* ws = nullptr;
  VL_HIP(noalloc_scratch(&ws));
  VL_HIP(contrastive_loss(emb, texts, n, dim, head == VL_HEAD_SOFTMAX ? 0 : 1, scale, bias, loss,
                          d_emb, d_texts, d_scale_bias, ws, static_cast<hipStream_t>(stream)));
  return VL_OK;
}

vl_status vl_bf16_round(const float* src, int64_t n, int32_t method, uint16_t* dst,
                        void* stream) {
  if (!src || !dst) return fail(VL_ERR_INVALID_ARG, "NULL pointer argument");
  if (n <= 0 || n % 2) return fail(VL_ERR_INVALID_ARG, "n must be positive and even");
  if (method != 0 && method != 1) return fail(VL_ERR_INVALID_ARG, "method must be 0 or 1");
  if (reinterpret_cast<uintptr_t>(src) % 8 || reinterpret_cast<uintptr_t>(dst) % 4)
    return fail(VL_ERR_INVALID_ARG, "src must be 8-byte and dst 4-byte aligned");
  VL_HIP(bf16_round(src, reinterpret_cast<bf16_t*>(dst), (size_t)n, method,
                    static_cast<hipStream_t>(stream)));
  return VL_OK;
}

vl_status vl_fp8_quantize_rows(const float* src, int32_t rows, int32_t cols, uint8_t* codes,
                               float* scales, void* stream) {
  if (!src || !codes || !scales) return fail(VL_ERR_INVALID_ARG, "NULL pointer argument");
  if (rows <= 0 || cols <= 0) return fail(VL_ERR_INVALID_ARG, "rows and cols must be > 0");
  VL_HIP(quantise_e4m3_rows(src, codes, scales, rows, cols, static_cast<hipStream_t>(stream)));
  return VL_OK;
}

vl_status vl_score(const float* emb, int32_t n_images, const float* texts, int32_t n_texts,
                   int32_t dim, vl_head head, float scale, float bias, float* scores,
                   int32_t* top1, void* stream) {
  if (!emb || !texts || !scores) return fail(VL_ERR_INVALID_ARG, "NULL pointer argument");
  if (n_images <= 0 || n_texts <= 0 || dim <= 0) return fail(VL_ERR_INVALID_ARG, "sizes must be > 0");
  if (dim % 4) return fail(VL_ERR_INVALID_ARG, "dim must be a multiple of 4");
  if (n_texts % 4) return fail(VL_ERR_INVALID_ARG, "n_texts must be a multiple of 4");
  if (head != VL_HEAD_SOFTMAX && head != VL_HEAD_SIGMOID) return fail(VL_ERR_INVALID_ARG, "unknown head");
  if (!std::isfinite(scale) || !std::isfinite(bias)) return fail(VL_ERR_INVALID_ARG, "scale/bias not finite");
  if (reinterpret_cast<uintptr_t>(emb) % 16 || reinterpret_cast<uintptr_t>(texts) % 16 ||
      reinterpret_cast<uintptr_t>(scores) % 16)
    return fail(VL_ERR_INVALID_ARG, "emb, texts and scores must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  EpiArgs e;
  e.out = scores;
  e.ldo = n_texts;
  e.alpha = scale;
  e.beta = bias;
  VL_HIP(gemm_f32_rows(emb, dim, texts, dim, n_images, n_texts, dim, OP_LOGITS, e, s));
  VL_HIP(score_rows(scores, top1, n_images, n_texts, head == VL_HEAD_SOFTMAX ? 0 : 1, s));
  return VL_OK;
}

}  // extern "C"

// ------------------------------------------------- attention on its own
namespace {

constexpr int kMaxAttnLen = 4096;  // longest sequence vl_attention accepts

// Descriptor blob of a vl_attention call: sequence descriptors, the
// 128-query work items, then the sequences that run K/V-resident (each part
// 16-byte aligned), as the encoder lays them out.  resident: whether
// sequences of 129 .. 640 tokens go to the resident kernel.
struct AttnPlan {
  std::vector<char> desc;
  size_t off_items = 0, off_res = 0;
  int n_items = 0, n_res = 0, res_tiles = 0;
  int64_t T = 0;
};

bool attention_plan(int32_t n, const int32_t* lens, bool resident, AttnPlan* ap,
                    std::string* why) {
  if (n <= 0 || n > kMaxItems) { *why = "n_seqs must be 1..65535"; return false; }
  if (!lens) { *why = "lengths is NULL"; return false; }
  std::vector<ImgDesc> seqs(n);
  std::vector<AttnItem> items;
  std::vector<int32_t> res;
  int64_t t = 0;
  for (int i = 0; i < n; ++i) {
    if (lens[i] < 1 || lens[i] > kMaxAttnLen) {
      *why = "sequence " + std::to_string(i) + " has length " + std::to_string(lens[i]) +
             ", not in 1..4096";
      return false;
    }
    ImgDesc& d = seqs[i];
    d.pix_off = 0;
    d.H = d.W = d.gh = d.gw = 0;
    d.tok_start = (int32_t)t;
    d.ntok = lens[i];
    if (resident && lens[i] > kResMinTokens && lens[i] <= 64 * kResMaxTiles) {
      res.push_back(i);
      ap->res_tiles = std::max(ap->res_tiles, (lens[i] + 63) / 64);
    } else {
      for (int q0 = 0; q0 < lens[i]; q0 += kAttnQ) items.push_back(AttnItem{i, q0});
    }
    t += lens[i];
  }
  if (t > (1LL << 24)) { *why = "more than 2^24 tokens"; return false; }
  auto a16 = [](size_t x) { return (x + 15) / 16 * 16; };
  ap->off_items = a16(sizeof(ImgDesc) * n);
  ap->off_res = a16(ap->off_items + sizeof(AttnItem) * items.size());
  ap->desc.assign(ap->off_res + sizeof(int32_t) * res.size(), 0);
  std::memcpy(ap->desc.data(), seqs.data(), sizeof(ImgDesc) * n);
  std::memcpy(ap->desc.data() + ap->off_items, items.data(), sizeof(AttnItem) * items.size());
  std::memcpy(ap->desc.data() + ap->off_res, res.data(), sizeof(int32_t) * res.size());
  ap->n_items = (int)items.size();
  ap->n_res = (int)res.size();
  ap->T = t;
  return true;
}

// The attention backward's descriptor region: sequences, then 64- and
// 128-token blocks (16-byte aligned); then, each 256-byte aligned, the
// log-sum-exp and D = rowsum(dO O) scratch [T, heads] FP32 and dO in BF16
// [T, heads * head_dim].
struct AttnBwdPlan {
  std::vector<char> desc;
  size_t off_items64 = 0, off_items128 = 0, off_lse = 0, off_dsum = 0, off_dob = 0, total = 0;
  int n_items64 = 0, n_items128 = 0;
  int64_t T = 0;
};

bool attention_bwd_plan(int32_t n, const int32_t* lens, int heads, int head_dim,
                        AttnBwdPlan* bp, std::string* why) {
  if (n <= 0 || n > kMaxItems) { *why = "n_seqs must be 1..65535"; return false; }
  if (!lens) { *why = "lengths is NULL"; return false; }
  std::vector<ImgDesc> seqs(n);
  std::vector<AttnItem> it64, it128;
  int64_t t = 0;
  for (int i = 0; i < n; ++i) {
    if (lens[i] < 1 || lens[i] > kMaxAttnLen) {
      *why = "sequence " + std::to_string(i) + " has length " + std::to_string(lens[i]) +
             ", not in 1..4096";
      return false;
    }
    ImgDesc& d = seqs[i];
    d.pix_off = 0;
    d.H = d.W = d.gh = d.gw = 0;
    d.tok_start = (int32_t)t;
    d.ntok = lens[i];
    for (int q0 = 0; q0 < lens[i]; q0 += 64) it64.push_back(AttnItem{i, q0});
    for (int q0 = 0; q0 < lens[i]; q0 += 128) it128.push_back(AttnItem{i, q0});
    t += lens[i];
  }
  if (t > (1LL << 24)) { *why = "more than 2^24 tokens"; return false; }
  auto a16 = [](size_t x) { return (x + 15) / 16 * 16; };
  bp->off_items64 = a16(sizeof(ImgDesc) * n);
  bp->off_items128 = a16(bp->off_items64 + sizeof(AttnItem) * it64.size());
  bp->desc.assign(bp->off_items128 + sizeof(AttnItem) * it128.size(), 0);
  std::memcpy(bp->desc.data(), seqs.data(), sizeof(ImgDesc) * n);
  std::memcpy(bp->desc.data() + bp->off_items64, it64.data(), sizeof(AttnItem) * it64.size());
  std::memcpy(bp->desc.data() + bp->off_items128, it128.data(),
              sizeof(AttnItem) * it128.size());
  bp->n_items64 = (int)it64.size();
  bp->n_items128 = (int)it128.size();
  bp->T = t;
  bp->off_lse = align_up(bp->desc.size());
  bp->off_dsum = bp->off_lse + align_up(4 * (size_t)t * heads);
  bp->off_dob = bp->off_dsum + align_up(4 * (size_t)t * heads);
  bp->total = bp->off_dob + align_up(2 * (size_t)t * heads * head_dim);
  return true;
}

}  // namespace

extern "C" {

size_t vl_attention_workspace_bytes(int32_t n_seqs, const int32_t* lengths) {
  AttnPlan ap;
  std::string why;
  if (!attention_plan(n_seqs, lengths, false, &ap, &why)) return 0;
  // an upper bound for every precision: all work items plus a resident list
  return align_up(ap.desc.size() + sizeof(int32_t) * (size_t)n_seqs + 16);
}

vl_status vl_attention(const void* qkv, vl_precision prec, const int32_t* lengths, int32_t n_seqs,
                       int32_t heads, int32_t head_dim, int32_t causal, void* out, void* ws,
                       size_t ws_bytes, void* stream) {
  if (!qkv || !out || !ws) return fail(VL_ERR_INVALID_ARG, "qkv, out or workspace is NULL");
  if (prec != VL_FP32 && prec != VL_BF16)
    return fail(VL_ERR_INVALID_ARG, "precision must be VL_FP32 or VL_BF16");
  if (heads < 1 || heads > 64) return fail(VL_ERR_INVALID_ARG, "heads must be 1..64");
  if (head_dim != 32 && head_dim != 64) return fail(VL_ERR_UNSUPPORTED, "head_dim must be 32 or 64");
  auto al = [](const void* p, uintptr_t k) { return reinterpret_cast<uintptr_t>(p) % k == 0; };
  if (!al(qkv, 16) || !al(out, 16) || !al(ws, kAlign))
    return fail(VL_ERR_INVALID_ARG, "qkv and out must be 16-byte, the workspace 256-byte aligned");
  AttnPlan ap;
  std::string why;
  const bool resident = prec == VL_BF16 && head_dim == 64 && causal == 0;
  if (!attention_plan(n_seqs, lengths, resident, &ap, &why)) return fail(VL_ERR_INVALID_ARG, why);
  const std::vector<char>& desc = ap.desc;
  if (ws_bytes < align_up(desc.size()))
    return fail(VL_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  {
    // Descriptors go up through a library-wide ring of pinned buffers.
    static std::mutex mu;
    static std::vector<Staging> ring(8);
    static size_t pos = 0;
    std::lock_guard<std::mutex> lk(mu);
    vl_status st = stage_copy(ring, pos, desc.data(), desc.size(), w, s);
    if (st != VL_OK) return st;
  }
  const ImgDesc* d_seqs = reinterpret_cast<const ImgDesc*>(w);
  const AttnItem* d_items = reinterpret_cast<const AttnItem*>(w + ap.off_items);
  if (prec == VL_BF16) {
    VL_HIP(attention_bf16(static_cast<const bf16_t*>(qkv), static_cast<bf16_t*>(out), d_seqs,
                          d_items, ap.n_items, heads, head_dim, causal != 0, s));
    VL_HIP(attention_bf16_resident(static_cast<const bf16_t*>(qkv), out, nullptr, false,
                                   (int)ap.T, d_seqs, reinterpret_cast<const int*>(w + ap.off_res),
                                   ap.n_res, ap.res_tiles, heads, head_dim, s));
  } else {
    VL_HIP(attention_f32(static_cast<const float*>(qkv), static_cast<float*>(out), d_seqs,
                         d_items, ap.n_items, heads, head_dim, causal != 0, s));
  }
  return VL_OK;
}

size_t vl_attention_backward_workspace_bytes(int32_t n_seqs, const int32_t* lengths,
                                             int32_t heads, int32_t head_dim) {
  if (heads < 1 || heads > 64 || (head_dim != 32 && head_dim != 64)) return 0;
  AttnBwdPlan bp;
  std::string why;
  if (!attention_bwd_plan(n_seqs, lengths, heads, head_dim, &bp, &why)) return 0;
  return bp.total;
}

vl_status vl_attention_backward(const void* qkv, const void* out, const float* d_out,
                                vl_precision prec, const int32_t* lengths, int32_t n_seqs,
                                int32_t heads, int32_t head_dim, void* d_qkv, void* ws,
                                size_t ws_bytes, void* stream) {
  if (!qkv || !out || !d_out || !d_qkv || !ws)
    return fail(VL_ERR_INVALID_ARG, "qkv, out, d_out, d_qkv or workspace is NULL");
  if (prec != VL_FP32 && prec != VL_BF16)
    return fail(VL_ERR_INVALID_ARG, "precision must be VL_FP32 or VL_BF16");
  if (heads < 1 || heads > 64) return fail(VL_ERR_INVALID_ARG, "heads must be 1..64");
  if (head_dim != 32 && head_dim != 64) return fail(VL_ERR_UNSUPPORTED, "head_dim must be 32 or 64");
  auto al = [](const void* p, uintptr_t k) { return reinterpret_cast<uintptr_t>(p) % k == 0; };
  if (!al(qkv, 16) || !al(out, 16) || !al(d_out, 16) || !al(d_qkv, 16) || !al(ws, kAlign))
    return fail(VL_ERR_INVALID_ARG,
                "qkv, out, d_out and d_qkv must be 16-byte, the workspace 256-byte aligned");
  AttnBwdPlan bp;
  std::string why;
  if (!attention_bwd_plan(n_seqs, lengths, heads, head_dim, &bp, &why))
    return fail(VL_ERR_INVALID_ARG, why);
  if (ws_bytes < bp.total) return fail(VL_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  {
    static std::mutex mu;
    static std::vector<Staging> ring(8);
    static size_t pos = 0;
    std::lock_guard<std::mutex> lk(mu);
    vl_status st = stage_copy(ring, pos, bp.desc.data(), bp.desc.size(), w, s);
    if (st != VL_OK) return st;
  }
  const bool bf = prec == VL_BF16;
  bf16_t* dob = reinterpret_cast<bf16_t*>(w + bp.off_dob);
  if (bf) VL_HIP(convert_bf16(d_out, dob, (size_t)bp.T * heads * head_dim, s));
  VL_HIP(attention_backward(qkv, out, bf, d_out, reinterpret_cast<const ImgDesc*>(w),
                            reinterpret_cast<const AttnItem*>(w + bp.off_items64), bp.n_items64,
                            reinterpret_cast<const AttnItem*>(w + bp.off_items128),
                            bp.n_items128, heads, head_dim, d_qkv,
                            reinterpret_cast<float*>(w + bp.off_lse),
                            reinterpret_cast<float*>(w + bp.off_dsum), s, false,
                            bf ? dob : nullptr));
  return VL_OK;
}

}  // extern "C"

// ------------------------------------------------ tuning table as JSON
namespace {

const char* kGemmOpNames[VL_N_GEMM_OPS] = {"patch_embed", "qkv_gemm", "oproj_gemm", "fc1_gemm",
                                           "fc2_gemm"};
const char* kPrecNames[4] = {"fp32", "bf16", "fp8w", "mxfp8"};

std::string device_arch(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');   // drop feature suffixes such as ":sramecc+:xnack-"
  return c == std::string::npos ? a : a.substr(0, c);
}

// A minimal JSON reader for the tuning file: objects, strings (no escapes
// beyond \" and \\), numbers, true / false / null.  Arrays are not used.
struct JVal {
  enum Kind { NUL, NUM, STR, OBJ, BOOL } kind = NUL;
  double num = 0;
  std::string str;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal* get(const char* k) const {
    for (const auto& kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

struct JParser {
  const std::string& s;
  size_t i = 0;
  explicit JParser(const std::string& t) : s(t) {}
  void ws() { while (i < s.size() && std::isspace((unsigned char)s[i])) ++i; }
  bool str(std::string* out) {
    ws();
    if (i >= s.size() || s[i] != '"') return false;
    ++i;
    out->clear();
    while (i < s.size() && s[i] != '"') {
      if (s[i] == '\\') {
        if (++i >= s.size()) return false;
        if (s[i] != '"' && s[i] != '\\' && s[i] != '/') return false;
      }
      out->push_back(s[i++]);
    }
    if (i >= s.size()) return false;
    ++i;
    return true;
  }
  bool value(JVal* v, int depth) {
    if (depth > 8) return false;
    ws();
    if (i >= s.size()) return false;
    const char c = s[i];
    if (c == '{') {
      ++i;
      v->kind = JVal::OBJ;
      ws();
      if (i < s.size() && s[i] == '}') { ++i; return true; }
      for (;;) {
        std::string k;
        if (!str(&k)) return false;
        ws();
        if (i >= s.size() || s[i] != ':') return false;
        ++i;
        JVal x;
        if (!value(&x, depth + 1)) return false;
        v->obj.emplace_back(k, std::move(x));
        ws();
        if (i < s.size() && s[i] == ',') { ++i; continue; }
        if (i < s.size() && s[i] == '}') { ++i; return true; }
        return false;
      }
    }
    if (c == '"') { v->kind = JVal::STR; return str(&v->str); }
    if (s.compare(i, 4, "true") == 0) { v->kind = JVal::BOOL; v->num = 1; i += 4; return true; }
    if (s.compare(i, 5, "false") == 0) { v->kind = JVal::BOOL; i += 5; return true; }
    if (s.compare(i, 4, "null") == 0) { v->kind = JVal::NUL; i += 4; return true; }
    const char* b = s.c_str() + i;
    char* e = nullptr;
    v->num = std::strtod(b, &e);
    if (e == b) return false;
    v->kind = JVal::NUM;
    i += (size_t)(e - b);
    return true;
  }
};

}  // namespace

extern "C" {

vl_status vl_model_save_tuning(const vl_model* m, const char* path) {
  if (!m || !path) return fail(VL_ERR_INVALID_ARG, "NULL argument");
  std::string j = "{\n  \"abi\": " + std::to_string(VL_ABI_VERSION) + ",\n";
  j += "  \"arch\": \"" + device_arch(m->device) + "\",\n";
  j += std::string("  \"precision\": \"") + kPrecNames[m->prec] + "\",\n";
  j += "  \"text\": " + std::string(m->text ? "true" : "false") + ",\n";
  j += "  \"width\": " + std::to_string(m->D) + ",\n  \"mlp\": " + std::to_string(m->F) +
       ",\n  \"patch_k\": " + std::to_string(m->Kpad) + ",\n";
  j += "  \"table\": {";
  for (int op = 0; op < VL_N_GEMM_OPS; ++op) {
    j += std::string(op ? ",\n" : "\n") + "    \"" + kGemmOpNames[op] + "\": {";
    bool first = true;
    for (int b = 0; b < VL_N_M_BUCKETS; ++b) {
      const int c = m->tuning[op][b];
      if (c < 0) continue;
      j += std::string(first ? "" : ", ") + "\"" + std::to_string(b) + "\": \"" + gemm_cfg_name(c) +
           "\"";
      first = false;
    }
    j += "}";
  }
  j += "\n  }\n}\n";
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(VL_ERR_INVALID_ARG, std::string("cannot write ") + path);
  const size_t n = std::fwrite(j.data(), 1, j.size(), f);
  const int rc = std::fclose(f);
  if (n != j.size() || rc != 0) return fail(VL_ERR_INVALID_ARG, std::string("cannot write ") + path);
  return VL_OK;
}

vl_status vl_model_load_tuning(vl_model* m, const char* path) {
  if (!m || !path) return fail(VL_ERR_INVALID_ARG, "NULL argument");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(VL_ERR_INVALID_ARG, std::string("cannot read ") + path);
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0 && text.size() < (1u << 20)) text.append(buf, n);
  std::fclose(f);
  JVal root;
  JParser ps(text);
  if (!ps.value(&root, 0) || root.kind != JVal::OBJ)
    return fail(VL_ERR_INVALID_ARG, std::string(path) + " is not a JSON object");
  auto num = [&](const char* k) { const JVal* v = root.get(k); return v && v->kind == JVal::NUM ? v->num : -1.0; };
  auto strv = [&](const char* k) { const JVal* v = root.get(k); return v && v->kind == JVal::STR ? v->str : std::string(); };
  const JVal* txt = root.get("text");
  const bool is_text = txt && txt->kind == JVal::BOOL && txt->num != 0;
  if ((int)num("abi") != VL_ABI_VERSION || strv("arch") != device_arch(m->device) ||
      strv("precision") != kPrecNames[m->prec] || is_text != m->text ||
      (int)num("width") != m->D || (int)num("mlp") != m->F || (int)num("patch_k") != m->Kpad)
    return fail(VL_ERR_INVALID_ARG, std::string(path) +
                                        " was tuned for another device, precision or model shape");
  const JVal* table = root.get("table");
  if (!table || table->kind != JVal::OBJ) return fail(VL_ERR_INVALID_ARG, "no \"table\" object");
  int32_t t[VL_N_GEMM_OPS][VL_N_M_BUCKETS];
  for (auto& row : t)
    for (auto& v : row) v = -1;
  for (const auto& kv : table->obj) {
    int op = -1;
    for (int k = 0; k < VL_N_GEMM_OPS; ++k)
      if (kv.first == kGemmOpNames[k]) op = k;
    if (op < 0 || kv.second.kind != JVal::OBJ)
      return fail(VL_ERR_INVALID_ARG, "unknown GEMM operation \"" + kv.first + "\"");
    for (const auto& e : kv.second.obj) {
      char* end = nullptr;
      const long b = std::strtol(e.first.c_str(), &end, 10);
      if (end == e.first.c_str() || *end || b < 0 || b >= VL_N_M_BUCKETS)
        return fail(VL_ERR_INVALID_ARG, "bad M bucket \"" + e.first + "\"");
      int id = -1;
      for (int c = 0; c < N_GEMM_CFGS; ++c)
        if (e.second.kind == JVal::STR && e.second.str == gemm_cfg_name(c)) id = c;
      if (id < 0) return fail(VL_ERR_INVALID_ARG, "unknown tile configuration in " + kv.first);
      t[op][b] = id;
    }
  }
  return vl_model_set_tuning(m, &t[0][0]);
}

}  // extern "C"

// ================================================= training through the tower
namespace {

// Workspace of a training forward + backward: the one-part encode plan, then
// per block the activations the backward reads, then the backward's scratch.
// Kept per block: input x, LN1 output, QKV, attention output, post-attention
// residual h, LN2 output, FC1 pre-activation z1 (FP32), the forward
// attention's log-sum-exp and (BF16 models) GELU(z1) as FC2 read it.
struct TrainLayer { size_t xin, y1, qkv, o, h, y2, z1, lse, g = 0; };
struct TrainPlan {
  Plan p;
  size_t off_items64 = 0;   // 64-token attention blocks (dK / dV), in the descriptor region
  int n_items64 = 0;
  size_t off_items128 = 0;  // 128-token attention blocks (dQ), after them
  int n_items128 = 0;
  int Tp = 0;               // T rounded up to 64 (K of the weight-gradient GEMMs)
  std::vector<TrainLayer> layers;
  size_t dX, dXb, gT, actT, dGf, dZ, dY, Wt, lse, dsum, part, pg, pb, de, zp, ppg, ppb, dwf;
  size_t dOb = 0;   // dO of the attention in BF16 (BF16 models)
  // The training forward as two halves of consecutive images on two streams
  // (VL_OPT_SPLIT, BF16): each half's descriptors (token starts relative to
  // the half) in the descriptor region, its rows / images at t0 / i0 of the
  // whole-batch buffers.  Empty: one pass over the batch.
  struct Half {
    int i0 = 0, n = 0, t0 = 0, T = 0, max_ntok = 0, n_items = 0, n_res = 0, res_tiles = 0;
    size_t off_imgs = 0, off_items = 0, off_res = 0;
  };
  std::vector<Half> halves;
  size_t off_split = 0;
  // The attention-pooling head: kept forward values (LN_f of every token,
  // its K/V projection, the head's rows) and backward scratch.
  struct Map {
    bool on = false;
    size_t yf = 0, kv = 0, dkv = 0, mo = 0, my = 0, mzl = 0, mz = 0, mh = 0;
    size_t dy = 0, dzl = 0, dO = 0, dq = 0, dhg = 0, hpre = 0, dh = 0, gtmp = 0, wt = 0;
  } map;
  size_t zscr = 0;  // pooled rows [n, D] (final LayerNorm scratch of the forward)
  size_t wsplit = 0, wsplit_bytes = 0;   // split-K partial products of the weight gradients
  size_t total = 0;
};

// Splits of a weight-gradient GEMM [M, N] over K = Tp (BF16 models): as many
// as keep the 256 x 256 tiles of all splits within half a round of 256 CUs,
// each split a multiple of 64 columns.  Every split adds an FP32 partial
// product to write and sum, and the weight gradients run on a second stream
// beside the input-gradient chain, which takes the other CUs.  Measured on
// MI355X at ViT-L/14@336, batch 32 (one box, training step): half a round
// 55.7 ms, a full round 56.5 ms, a quarter round 68 ms; two splits for every
// product 55.3 against 54.9 ms for half a round.  Returns (splits, columns
// per split).
std::pair<int, int> wgrad_splits(int M, int N, int Tp) {
  const int tiles = ((M + 255) / 256) * ((N + 255) / 256);
  int want = std::max(1, std::min(128 / tiles, Tp / 64));
  const int kc = ((Tp + want - 1) / want + 63) / 64 * 64;
  return {(Tp + kc - 1) / kc, kc};
}

bool make_train_plan(const vl_model* m, int32_t n, const int32_t* hs, const int32_t* ws,
                     TrainPlan* tp, std::string* why) {
  if (m->text) { *why = "training covers the image tower"; return false; }
  if (m->prec != VL_FP32 && m->prec != VL_BF16) {
    *why = "training runs in VL_FP32 or VL_BF16";
    return false;
  }
  const bool map = m->cfg.pool == VL_POOL_MAP;
  if (map && m->hd > 64) { *why = "training the pooling head needs head width <= 64"; return false; }
  if (!make_plan(m, n, hs, ws, &tp->p, why, /*one_part=*/true)) return false;
  for (int i = 0; i < n; ++i)
    if (hs[i] / m->P != m->g0 || ws[i] / m->P != m->g0) {
      *why = "image " + std::to_string(i) + ": training needs the base patch grid (" +
             std::to_string(m->g0) + " x " + std::to_string(m->g0) + ")";
      return false;
    }
  Plan& p = tp->p;
  // (2^20 tokens: the transposes' grid spans T / 32 rows of workgroups)
  if (p.T > (1 << 20)) { *why = "training batch exceeds 2^20 tokens"; return false; }
  // 64- and 128-token blocks of every image for the attention backward
  std::vector<AttnItem> it, it2;
  const ImgDesc* imgs = reinterpret_cast<const ImgDesc*>(p.desc.data() + p.parts[0].off_imgs);
  for (int i = 0; i < n; ++i) {
    for (int t0 = 0; t0 < imgs[i].ntok; t0 += 64) it.push_back(AttnItem{i, t0});
    for (int t0 = 0; t0 < imgs[i].ntok; t0 += 128) it2.push_back(AttnItem{i, t0});
  }
  tp->n_items64 = (int)it.size();
  tp->off_items64 = (p.desc_bytes + 15) / 16 * 16;
  tp->n_items128 = (int)it2.size();
  tp->off_items128 = tp->off_items64 + sizeof(AttnItem) * it.size();
  size_t new_desc = tp->off_items128 + sizeof(AttnItem) * it2.size();
  // Two halves for the forward: the split planner's parts, their descriptor
  // blob appended here.
  Plan sp;
  std::string why2;
  tp->halves.clear();
  if (m->prec == VL_BF16 && !map && make_plan(m, n, hs, ws, &sp, &why2) &&
      sp.parts.size() == 2) {
    const size_t base = (new_desc + 15) / 16 * 16;
    int t0 = 0;
    for (const Part& q : sp.parts) {
      TrainPlan::Half h;
      h.i0 = q.i0; h.n = q.n; h.t0 = t0; h.T = q.T; h.max_ntok = q.max_ntok;
      h.n_items = q.n_items; h.n_res = q.n_res; h.res_tiles = q.res_tiles;
      h.off_imgs = base + q.off_imgs; h.off_items = base + q.off_items;
      h.off_res = base + q.off_res;
      tp->halves.push_back(h);
      t0 += q.T;
    }
    tp->off_split = base;
    new_desc = base + sp.desc_bytes;
  }
  if (align_up(new_desc) > align_up(p.desc_bytes)) {
    // the activation regions start after the descriptor region: move them
    const size_t shift = align_up(new_desc) - align_up(p.desc_bytes);
    for (Part& q : p.parts) {
      q.off_tok += shift; q.off_X += shift; q.off_Y += shift; q.off_QH += shift; q.off_E += shift;
    }
    p.total += shift;
  }
  p.desc.resize(new_desc, 0);
  std::memcpy(p.desc.data() + tp->off_items64, it.data(), sizeof(AttnItem) * it.size());
  std::memcpy(p.desc.data() + tp->off_items128, it2.data(), sizeof(AttnItem) * it2.size());
  if (!tp->halves.empty()) std::memcpy(p.desc.data() + tp->off_split, sp.desc.data(), sp.desc_bytes);
  p.desc_bytes = new_desc;

  const size_t T = p.T, D = m->D, F = m->F, es = m->prec == VL_FP32 ? 4 : 2;
  const size_t Tp = (T + 63) / 64 * 64;
  tp->Tp = (int)Tp;
  size_t off = p.total;
  auto take = [&](size_t bytes) { const size_t r = off; off += align_up(bytes); return r; };
  tp->layers.resize(m->L);
  for (TrainLayer& l : tp->layers) {
    l.xin = take(4 * T * D); l.y1 = take(es * T * D); l.qkv = take(es * 3 * T * D);
    l.o = take(es * T * D); l.h = take(4 * T * D); l.y2 = take(es * T * D); l.z1 = take(4 * T * F);
    l.lse = take(4 * T * m->heads);   // the forward attention's log-sum-exp (BF16)
    if (es == 2) l.g = take(2 * T * F);
  }
  const size_t wide = std::max<size_t>({3 * D, F, (size_t)m->Kpad});
  tp->dX = take(4 * T * D);
  tp->dXb = es == 2 ? take(es * T * D) : tp->dX;
  if (es == 2) tp->dOb = take(es * T * D);
  tp->zscr = take(4 * (size_t)n * D);
  if (map) {
    TrainPlan::Map& mp = tp->map;
    mp.on = true;
    mp.yf = take(es * T * D); mp.kv = take(es * T * 2 * D); mp.dkv = take(es * T * 2 * D);
    mp.mo = take(4 * n * D); mp.my = take(4 * n * D); mp.mzl = take(4 * n * D);
    mp.mz = take(4 * n * D); mp.mh = take(4 * n * F);
    mp.dy = take(4 * n * D); mp.dzl = take(4 * n * D); mp.dO = take(4 * n * D);
    mp.dq = take(4 * n * D); mp.dhg = take(4 * n * F); mp.hpre = take(4 * n * F);
    mp.dh = take(4 * n * F); mp.gtmp = take(4 * n * F);
    mp.wt = take(4 * std::max(F * D, D * D));
  }
  tp->gT = take(es * std::max<size_t>(3 * D, F) * Tp);
  tp->actT = take(es * std::max<size_t>({D, F, (size_t)m->Kpad}) * Tp);
  tp->dGf = take(4 * T * F);
  tp->dZ = take(es * T * std::max<size_t>(3 * D, F));
  tp->dY = take(4 * T * D);
  tp->Wt = take(es * std::max<size_t>(3 * D * D, F * D));
  tp->lse = take(4 * T * m->heads);
  tp->dsum = take(4 * T * m->heads);
  tp->part = take(4 * ((T + kColRows - 1) / kColRows) * wide);
  tp->pg = take(4 * ((T + kLnRows - 1) / kLnRows) * D);
  tp->pb = take(4 * ((T + kLnRows - 1) / kLnRows) * D);
  tp->de = take(4 * (size_t)n * m->Pd);
  tp->zp = take(4 * (size_t)n * D);
  tp->ppg = take(4 * (size_t)n * D);
  tp->ppb = take(4 * (size_t)n * D);
  tp->dwf = take(4 * D * m->Kpad);
  if (es == 2) {
    size_t mx = 0;
    const size_t shapes[5][2] = {{D, F}, {F, D}, {D, D}, {3 * D, D}, {D, (size_t)m->Kpad}};
    for (const auto& sh : shapes) {
      const auto sp = wgrad_splits((int)sh[0], (int)sh[1], (int)Tp);
      if (sp.first > 1) mx = std::max(mx, (size_t)sp.first * sh[0] * sh[1] * 4);
    }
    tp->wsplit_bytes = mx;
    if (mx) tp->wsplit = take(mx);
  }
  tp->total = off;
  return true;
}

std::string train_key(const TrainPlan& tp, const void* pix, const void* ws, size_t ws_bytes) {
  std::string k;
  auto put = [&](const void* v, size_t b) { k.append(static_cast<const char*>(v), b); };
  put(&pix, sizeof pix); put(&ws, sizeof ws); put(&ws_bytes, sizeof ws_bytes);
  put(tp.p.hw.data(), sizeof(int32_t) * tp.p.hw.size());
  return k;
}

// FP32 product C[M, N] = A[M, K] . B[N, K]^T in the model's arithmetic (FP32
// FMA, or BF16 operands with FP32 accumulation on the MFMA kernel).
vl_status gemm_into_f32(const vl_model* m, const void* A, int lda, const void* B, int ldb, int M,
                        int N, int K, float* out, int ldo, hipStream_t s,
                        bf16_t* copy_bf16 = nullptr) {
  EpiArgs e;
  e.out = out; e.ldo = ldo; e.alpha = 1.f; e.beta = 0.f;
  e.out2 = m->prec == VL_FP32 ? nullptr : copy_bf16;   // BF16 copy of out (BF16 models)
  if (m->prec == VL_FP32)
    VL_HIP(gemm_f32(static_cast<const float*>(A), lda, static_cast<const float*>(B), ldb, M, N, K,
                    OP_LOGITS, e, s));
  else
    VL_HIP(gemm_bf16(static_cast<const bf16_t*>(A), lda, B, ldb, false, M, N, K, OP_LOGITS, -1, e,
                     s));
  return VL_OK;
}

// The training forward: the encoder's kernel sequence, keeping each block's
// input, LayerNorm outputs, Q/K/V, attention output, residual after
// attention, FC1 pre-activation and (BF16) GELU output.  Every kernel and its
// arithmetic is the inference forward's, so the embeddings agree with
// vl_encode_images bitwise.
//
// A run of consecutive images of a training batch: its rows t0 .. t0+T-1
// and images i0 .. i0+n-1 of the whole-batch buffers, with descriptors
// whose token starts are relative to t0.
struct FwdRange {
  int i0 = 0, n = 0, t0 = 0, T = 0, max_ntok = 0, n_items = 0, n_res = 0, res_tiles = 0;
  const ImgDesc* imgs = nullptr;
  const AttnItem* items = nullptr;
  const int* res = nullptr;
};

vl_status train_forward_range(vl_model* m, const TrainPlan& tp, const float* pix, float* emb,
                              char* ws, const FwdRange& r, hipStream_t s) {
  const Part& p = tp.p.parts[0];
  const bool f32 = m->prec == VL_FP32;
  const size_t es = f32 ? 4 : 2;
  const int T = r.T, D = m->D, F = m->F, t0 = r.t0;
  const float eps = m->cfg.ln_eps;
  int2* tok = reinterpret_cast<int2*>(ws + p.off_tok) + t0;
  float* X = reinterpret_cast<float*>(ws + p.off_X) + (size_t)t0 * D;
  void* QH = ws + p.off_QH + es * (size_t)t0 * m->Kpad;   // this range's patch rows
  // The residual stream is written straight into the kept per-block
  // buffers: block l reads its input from xin_l, the output projection
  // writes h_l = xin_l + ..., FC2 writes xin_{l+1} = h_l + ... (X after the
  // last block), so nothing is copied.
  auto xin_of = [&](int l) {
    return l < m->L ? reinterpret_cast<float*>(ws + tp.layers[l].xin) + (size_t)t0 * D : X;
  };
  EpiArgs pe;
  pe.bias = m->patch_b; pe.out = xin_of(0); pe.ldo = D; pe.tok_info = tok; pe.imgs = r.imgs;
  pe.cls = m->cls; pe.pos = m->pos; pe.base_grid = m->g0;
  VL_HIP(im2col(pix, r.imgs, r.n, r.max_ntok, m->cfg.channels, m->P, m->Kpad, QH, !f32, tok, s));
  if (f32)
    VL_HIP(gemm_f32(static_cast<const float*>(QH), m->Kpad, static_cast<const float*>(m->patch_w),
                    m->Kpad, T, D, m->Kpad, OP_PATCH, pe, s));
  else
    VL_HIP(gemm_bf16(static_cast<const bf16_t*>(QH), m->Kpad, m->patch_w, m->Kpad, false, T, D,
                     m->Kpad, OP_PATCH, gemm_cfg_for(m, 0, T), pe, s));
  for (int l = 0; l < m->L; ++l) {
    const Layer& ly = m->layers[l];
    const TrainLayer& sv = tp.layers[l];
    void* y1 = ws + sv.y1 + es * (size_t)t0 * D;
    void* qkv = ws + sv.qkv + es * (size_t)t0 * 3 * D;
    void* o = ws + sv.o + es * (size_t)t0 * D;
    void* y2 = ws + sv.y2 + es * (size_t)t0 * D;
    float* z1 = reinterpret_cast<float*>(ws + sv.z1) + (size_t)t0 * F;
    float* xin = xin_of(l);
    float* hb = reinterpret_cast<float*>(ws + sv.h) + (size_t)t0 * D;
    VL_HIP(layernorm_rows(xin, ly.ln1_g, ly.ln1_b, eps, y1, !f32, T, D, s));
    EpiArgs e1; e1.bias = ly.qkv_b; e1.out = qkv; e1.ldo = 3 * D;
    EpiArgs e2; e2.bias = ly.o_b; e2.out = hb; e2.resid_in = xin; e2.ldo = D;
    EpiArgs e3; e3.bias = ly.fc1_b; e3.out = z1; e3.ldo = F;
    EpiArgs e4; e4.bias = ly.fc2_b; e4.out = xin_of(l + 1); e4.resid_in = hb; e4.ldo = D;
    if (f32) {
      VL_HIP(gemm_f32(static_cast<const float*>(y1), D, static_cast<const float*>(ly.qkv_w), D, T,
                      3 * D, D, OP_QKV, e1, s));
      VL_HIP(attention_f32(static_cast<const float*>(qkv), static_cast<float*>(o), r.imgs, r.items,
                           r.n_items, m->heads, m->hd, false, s));
      VL_HIP(gemm_f32(static_cast<const float*>(o), D, static_cast<const float*>(ly.o_w), D, T, D,
                      D, OP_OPROJ, e2, s));
    } else {
      VL_HIP(gemm_bf16(static_cast<const bf16_t*>(y1), D, ly.qkv_w, D, false, T, 3 * D, D, OP_QKV,
                       gemm_cfg_for(m, 1, T), e1, s));
      float* lse = reinterpret_cast<float*>(ws + sv.lse) + (size_t)t0 * m->heads;
      VL_HIP(attention_bf16(static_cast<const bf16_t*>(qkv), static_cast<bf16_t*>(o), r.imgs,
                            r.items, r.n_items, m->heads, m->hd, false, s, nullptr, lse));
      VL_HIP(attention_bf16_resident(static_cast<const bf16_t*>(qkv), o, nullptr, false, T, r.imgs,
                                     r.res, r.n_res, r.res_tiles, m->heads, m->hd, s, nullptr,
                                     lse));
      VL_HIP(gemm_bf16(static_cast<const bf16_t*>(o), D, ly.o_w, D, false, T, D, D, OP_OPROJ,
                       gemm_cfg_for(m, 2, T), e2, s));
    }
    VL_HIP(layernorm_rows(hb, ly.ln2_g, ly.ln2_b, eps, y2, !f32, T, D, s));
    if (f32) {
      VL_HIP(gemm_f32(static_cast<const float*>(y2), D, static_cast<const float*>(ly.fc1_w), D, T,
                      F, D, OP_FC1_PRE, e3, s));
      VL_HIP(gelu_forward(z1, QH, false, (size_t)T * F, s));
      VL_HIP(gemm_f32(static_cast<const float*>(QH), F, static_cast<const float*>(ly.fc2_w), F, T,
                      D, F, OP_FC2, e4, s));
    } else {
      // GELU(z1) in BF16 from the same epilogue, kept for the backward
      bf16_t* g = reinterpret_cast<bf16_t*>(ws + sv.g) + (size_t)t0 * F;
      e3.out2 = g;
      VL_HIP(gemm_bf16(static_cast<const bf16_t*>(y2), D, ly.fc1_w, D, false, T, F, D, OP_FC1_PRE,
                       gemm_cfg_for(m, 3, T), e3, s));
      VL_HIP(gemm_bf16(g, F, ly.fc2_w, F, false, T, D, F, OP_FC2, gemm_cfg_for(m, 4, T), e4, s));
    }
  }
  if (tp.map.on) {
    // Attention-pooling head, as vl_encode_images runs it, keeping LN_f of
    // every token, their K / V, and the head's attention output o, its
    // output projection y, LN(y), the MLP activation and the head output.
    const TrainPlan::Map& mp = tp.map;
    auto fp = [&](size_t off) { return reinterpret_cast<float*>(ws + off); };
    void* yf = ws + mp.yf;
    void* kv = ws + mp.kv;
    float* e = reinterpret_cast<float*>(ws + p.off_E);
    VL_HIP(layernorm_rows(X, m->lnf_g, m->lnf_b, eps, yf, !f32, T, D, s));
    EpiArgs ekv;
    ekv.bias = m->map_kv_b; ekv.out = kv; ekv.ldo = 2 * D;
    if (f32)
      VL_HIP(gemm_f32(static_cast<const float*>(yf), D, static_cast<const float*>(m->map_kv_w), D,
                      T, 2 * D, D, OP_QKV, ekv, s));
    else
      VL_HIP(gemm_bf16(static_cast<const bf16_t*>(yf), D, m->map_kv_w, D, false, T, 2 * D, D,
                       OP_QKV, -1, ekv, s));
    VL_HIP(map_attention(kv, !f32, m->map_q, r.imgs, r.n, m->heads, m->hd, fp(mp.mo), s));
    EpiArgs e1; e1.bias = m->map_o_b; e1.out = fp(mp.my); e1.ldo = D;
    VL_HIP(gemm_f32_rows(fp(mp.mo), D, m->map_o_w, D, r.n, D, D, OP_QKV, e1, s));
    VL_HIP(layernorm_rows(fp(mp.my), m->map_ln_g, m->map_ln_b, eps, fp(mp.mzl), false, r.n, D,
                          s));
    EpiArgs e2; e2.bias = m->map_fc1_b; e2.out = fp(mp.mh); e2.ldo = F;
    VL_HIP(gemm_f32_rows(fp(mp.mzl), D, m->map_fc1_w, D, r.n, F, D, OP_FC1, e2, s));
    VL_HIP(copy_f32(fp(mp.my), fp(mp.mz), (size_t)r.n * D, s));
    EpiArgs e3; e3.bias = m->map_fc2_b; e3.out = fp(mp.mz); e3.ldo = D;
    VL_HIP(gemm_f32_rows(fp(mp.mh), F, m->map_fc2_w, F, r.n, D, F, OP_FC2, e3, s));
    EpiArgs e4; e4.out = e; e4.ldo = m->Pd;
    VL_HIP(gemm_f32_rows(fp(mp.mz), D, m->proj, D, r.n, m->Pd, D, OP_LOGITS, e4, s));
    VL_HIP(l2_normalise_rows(e, emb, r.n, m->Pd, s));
    return VL_OK;
  }
  VL_HIP(pool_project(X, r.imgs, r.n, m->lnf_g, m->lnf_b, eps, m->proj, D, m->Pd, false,
                      reinterpret_cast<float*>(ws + tp.zscr) + (size_t)r.i0 * D,
                      reinterpret_cast<float*>(ws + p.off_E) + (size_t)r.i0 * m->Pd,
                      emb + (size_t)r.i0 * m->Pd, s));
  return VL_OK;
}

// The training forward: one pass over the batch, or its two halves on the
// caller's stream and the model's side stream (forked after everything
// before this call on s, joined back into s, also after an error).  Every
// kernel works per token row or per image in a fixed order, so the halves
// compute the same bits as one pass.
vl_status run_train_forward(vl_model* m, const TrainPlan& tp, const float* pix, float* emb,
                            char* ws, hipStream_t s) {
  const Part& p = tp.p.parts[0];
  if (tp.halves.size() != 2) {
    FwdRange r;
    r.n = p.n; r.T = p.T; r.max_ntok = p.max_ntok; r.n_items = p.n_items; r.n_res = p.n_res;
    r.res_tiles = p.res_tiles;
    r.imgs = reinterpret_cast<const ImgDesc*>(ws + p.off_imgs);
    r.items = reinterpret_cast<const AttnItem*>(ws + p.off_items);
    r.res = reinterpret_cast<const int*>(ws + p.off_res);
    return train_forward_range(m, tp, pix, emb, ws, r, s);
  }
  if (!m->side) VL_HIP(hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking));
  if (!m->ev_fork) VL_HIP(hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming));
  if (!m->ev_join) VL_HIP(hipEventCreateWithFlags(&m->ev_join, hipEventDisableTiming));
  VL_HIP(hipEventRecord(m->ev_fork, s));
  VL_HIP(hipStreamWaitEvent(m->side, m->ev_fork, 0));
  vl_status st = VL_OK;
  for (int k = 0; k < 2 && st == VL_OK; ++k) {
    const TrainPlan::Half& h = tp.halves[k];
    FwdRange r;
    r.i0 = h.i0; r.n = h.n; r.t0 = h.t0; r.T = h.T; r.max_ntok = h.max_ntok;
    r.n_items = h.n_items; r.n_res = h.n_res; r.res_tiles = h.res_tiles;
    r.imgs = reinterpret_cast<const ImgDesc*>(ws + h.off_imgs);
    r.items = reinterpret_cast<const AttnItem*>(ws + h.off_items);
    r.res = reinterpret_cast<const int*>(ws + h.off_res);
    st = train_forward_range(m, tp, pix, emb, ws, r, k == 0 ? s : m->side);
  }
  if (hipEventRecord(m->ev_join, m->side) == hipSuccess)
    (void)hipStreamWaitEvent(s, m->ev_join, 0);
  return st;
}

// Offsets (floats) of every tensor in the FP32 weight blob, hence in the
// gradient blob (the same layout).
struct BlobOffsets {
  size_t patch_w, patch_b, cls, pos, lnf_g, lnf_b, proj;
  struct M { size_t probe, q_w, q_b, kv_w, kv_b, o_w, o_b, ln_g, ln_b, fc1_w, fc1_b, fc2_w, fc2_b; };
  M map{};   // attention-pooling head (pool = MAP)
  struct L { size_t ln1_g, ln1_b, qkv_w, qkv_b, o_w, o_b, ln2_g, ln2_b, fc1_w, fc1_b, fc2_w, fc2_b; };
  std::vector<L> layers;
};

BlobOffsets blob_offsets(const vl_model* m) {
  BlobOffsets b;
  const size_t D = m->D, F = m->F;
  size_t o = 0;
  auto take = [&](size_t n) { const size_t r = o; o += n; return r; };
  b.patch_w = take(D * m->Kpe); b.patch_b = take(D); b.cls = take(D);
  b.pos = take((1 + (size_t)m->g0 * m->g0) * D);
  b.layers.resize(m->L);
  for (auto& l : b.layers) {
    l.ln1_g = take(D); l.ln1_b = take(D); l.qkv_w = take(3 * D * D); l.qkv_b = take(3 * D);
    l.o_w = take(D * D); l.o_b = take(D); l.ln2_g = take(D); l.ln2_b = take(D);
    l.fc1_w = take(F * D); l.fc1_b = take(F); l.fc2_w = take(D * F); l.fc2_b = take(D);
  }
  b.lnf_g = take(D); b.lnf_b = take(D);
  if (!m->text && m->cfg.pool == VL_POOL_MAP) {
    BlobOffsets::M& q = b.map;
    q.probe = take(D); q.q_w = take(D * D); q.q_b = take(D); q.kv_w = take(2 * D * D);
    q.kv_b = take(2 * D); q.o_w = take(D * D); q.o_b = take(D); q.ln_g = take(D); q.ln_b = take(D);
    q.fc1_w = take(F * D); q.fc1_b = take(F); q.fc2_w = take(D * F); q.fc2_b = take(D);
  }
  b.proj = take((size_t)m->Pd * D);
  return b;
}

// Weight gradient out [M, N] = A [M, Tp] . B [N, Tp]^T: in BF16 models a
// split-K product (partials in the workspace, added in split order), so the
// few output tiles of these GEMMs are spread over the CUs.
vl_status wgrad_gemm(const vl_model* m, const TrainPlan& tp, char* ws, const void* A,
                     const void* B, int M, int N, float* out, hipStream_t s) {
  const int Tp = tp.Tp;
  if (m->prec == VL_FP32) return gemm_into_f32(m, A, Tp, B, Tp, M, N, Tp, out, N, s);
  const auto sp = wgrad_splits(M, N, Tp);
  if (sp.first <= 1 || (size_t)sp.first * M * N * 4 > tp.wsplit_bytes)
    return gemm_into_f32(m, A, Tp, B, Tp, M, N, Tp, out, N, s);
  float* part = reinterpret_cast<float*>(ws + tp.wsplit);
  EpiArgs e;
  e.out = part; e.ldo = N; e.alpha = 1.f; e.beta = 0.f;
  e.kc = sp.second;
  e.zstride = (size_t)M * N;
  VL_HIP(gemm_bf16(static_cast<const bf16_t*>(A), Tp, B, Tp, false, M, N, Tp, OP_LOGITS,
                   CFG_DL_256x256_W2x4, e, s));
  VL_HIP(sum_splits(part, sp.first, (size_t)M * N, out, s));
  return VL_OK;
}

// The same weight gradient from token-major BF16 operands: out [M, N] =
// A^T B with A [T, lda] (columns 0..M-1) and B [T, ldb] (columns 0..N-1),
// the token rows T..Tp-1 read as zero; same splits, same partial sums.
vl_status wgrad_gemm_km(const TrainPlan& tp, char* ws, const void* A, int lda, const void* B,
                        int ldb, int M, int N, float* out, hipStream_t s) {
  const int Tp = tp.Tp, T = tp.p.T;
  auto sp = wgrad_splits(M, N, Tp);
  EpiArgs e;
  e.alpha = 1.f; e.beta = 0.f;
  e.ldo = N;
  const bool split = sp.first > 1 && (size_t)sp.first * M * N * 4 <= tp.wsplit_bytes;
  float* part = reinterpret_cast<float*>(ws + tp.wsplit);
  e.out = split ? part : out;
  e.kc = split ? sp.second : Tp;
  e.zstride = (size_t)M * N;
  VL_HIP(gemm_bf16_kmajor(static_cast<const bf16_t*>(A), lda, static_cast<const bf16_t*>(B), ldb,
                          M, N, Tp, T, e, s));
  if (split) VL_HIP(sum_splits(part, sp.first, (size_t)M * N, out, s));
  return VL_OK;
}

// Backward of the attention-pooling head and of the final LayerNorm over
// every token (the chain rule of the head's forward, as the oracle writes
// it): L2 and projection, the head's MLP residual and LayerNorm, its output
// projection, the one-query attention, the query (probe) and K / V
// projections, then LN_f; leaves dL/dX of every token in dX.  The head's
// small products (rows of n images) run on the FP32 row GEMM against
// transposed weights, the K / V projection's on the block GEMMs.
vl_status map_head_backward(vl_model* m, const TrainPlan& tp, char* ws, const float* demb,
                            float* grads, const BlobOffsets& bo, hipStream_t s) {
  const Part& p = tp.p.parts[0];
  const TrainPlan::Map& mp = tp.map;
  const bool f32 = m->prec == VL_FP32, bf = !f32;
  const int T = p.T, n = p.n, D = m->D, F = m->F, Pd = m->Pd, Tp = tp.Tp;
  const float eps = m->cfg.ln_eps;
  const ImgDesc* d_imgs = reinterpret_cast<const ImgDesc*>(ws + p.off_imgs);
  auto fp = [&](size_t off) { return reinterpret_cast<float*>(ws + off); };
  auto G = [&](size_t off) { return grads + off; };
  float* part = fp(tp.part);
  float* pg = fp(tp.pg);
  float* pb = fp(tp.pb);
  float* wt = fp(mp.wt);
  float* dz = fp(tp.zp);   // dL/d(head output) [n, D]
  const BlobOffsets::M& g = bo.map;
  auto rows = [&](const float* A, int lda, const float* B, int ldb, int M, int N, int K,
                  float* out) -> vl_status {
    EpiArgs e;
    e.out = out; e.ldo = N; e.alpha = 1.f; e.beta = 0.f;
    VL_HIP(gemm_f32_rows(A, lda, B, ldb, M, N, K, OP_LOGITS, e, s));
    return VL_OK;
  };
  vl_status st;
  // e = W_p z, e_hat = e / |e|
  VL_HIP(l2proj_backward(fp(p.off_E), demb, m->proj, n, D, Pd, fp(tp.de), dz, s));
  VL_HIP(outer_sum(fp(tp.de), fp(mp.mz), n, Pd, D, G(bo.proj), s));
  // z = y + GELU(LN(y) W1^T + b1) W2^T + b2
  VL_HIP(copy_f32(dz, fp(mp.dy), (size_t)n * D, s));
  VL_HIP(outer_sum(dz, fp(mp.mh), n, D, F, G(g.fc2_w), s));
  VL_HIP(colsum(dz, false, n, D, D, nullptr, part, G(g.fc2_b), s));
  VL_HIP(transpose_rows(m->map_fc2_w, false, D, F, F, wt, false, D, s));          // W2^T [F, D]
  if ((st = rows(dz, D, wt, D, n, F, D, fp(mp.dhg))) != VL_OK) return st;
  {
    EpiArgs e;
    e.bias = m->map_fc1_b; e.out = fp(mp.hpre); e.ldo = F;                      // pre-activation
    VL_HIP(gemm_f32_rows(fp(mp.mzl), D, m->map_fc1_w, D, n, F, D, OP_QKV, e, s));
  }
  VL_HIP(gelu_backward(fp(mp.dhg), fp(mp.hpre), fp(mp.dh), fp(mp.gtmp), false, (size_t)n * F, s));
  VL_HIP(outer_sum(fp(mp.dh), fp(mp.mzl), n, F, D, G(g.fc1_w), s));
  VL_HIP(colsum(fp(mp.dh), false, n, F, F, nullptr, part, G(g.fc1_b), s));
  VL_HIP(transpose_rows(m->map_fc1_w, false, F, D, D, wt, false, F, s));          // W1^T [D, F]
  if ((st = rows(fp(mp.dh), F, wt, F, n, D, F, fp(mp.dzl))) != VL_OK) return st;
  VL_HIP(layernorm_backward(fp(mp.my), m->map_ln_g, fp(mp.dzl), eps, fp(mp.dy), n, D, pg, pb,
                            G(g.ln_g), G(g.ln_b), s));
  // y = o W_o^T + b_o
  VL_HIP(outer_sum(fp(mp.dy), fp(mp.mo), n, D, D, G(g.o_w), s));
  VL_HIP(colsum(fp(mp.dy), false, n, D, D, nullptr, part, G(g.o_b), s));
  VL_HIP(transpose_rows(m->map_o_w, false, D, D, D, wt, false, D, s));            // W_o^T
  if ((st = rows(fp(mp.dy), D, wt, D, n, D, D, fp(mp.dO))) != VL_OK) return st;
  // one query per head over each image's K / V
  VL_HIP(map_attention_backward(ws + mp.kv, bf, m->map_q, fp(mp.mo), fp(mp.dO), d_imgs, n,
                                p.max_ntok, m->heads, m->hd, ws + mp.dkv, fp(mp.dq), s));
  // q = probe W_q^T + b_q, shared by every image: dq summed over images
  VL_HIP(colsum(fp(mp.dq), false, n, D, D, nullptr, part, G(g.q_b), s));
  VL_HIP(outer_sum(G(g.q_b), m->map_probe, 1, D, D, G(g.q_w), s));
  VL_HIP(transpose_rows(m->map_q_w, false, D, D, D, wt, false, D, s));            // W_q^T
  if ((st = rows(G(g.q_b), D, wt, D, 1, D, D, G(g.probe))) != VL_OK) return st;
  // [K | V] = LN_f(x) W_kv^T + b_kv over every token
  void* gT = ws + tp.gT;
  void* actT = ws + tp.actT;
  VL_HIP(colsum(ws + mp.dkv, bf, T, 2 * D, 2 * D, nullptr, part, G(g.kv_b), s));
  VL_HIP(transpose_rows(ws + mp.dkv, bf, T, 2 * D, 2 * D, gT, bf, Tp, s));
  VL_HIP(transpose_rows(ws + mp.yf, bf, T, D, D, actT, bf, Tp, s));
  if ((st = wgrad_gemm(m, tp, ws, gT, actT, 2 * D, D, G(g.kv_w), s)) != VL_OK) return st;
  VL_HIP(transpose_rows(m->map_kv_w, bf, 2 * D, D, D, ws + tp.Wt, bf, 2 * D, s));  // W_kv^T
  float* dY = fp(tp.dY);
  if ((st = gemm_into_f32(m, ws + mp.dkv, 2 * D, ws + tp.Wt, 2 * D, T, D, 2 * D, dY, D, s)) !=
      VL_OK)
    return st;
  // LN_f on every token: dX (zero) += LN_f'(X) dY
  VL_HIP(layernorm_backward(reinterpret_cast<const float*>(ws + p.off_X), m->lnf_g, dY, eps,
                            fp(tp.dX), T, D, pg, pb, G(bo.lnf_g), G(bo.lnf_b), s));
  return VL_OK;
}

// Events of the overlapped backward (indices into vl_model::tev): recorded on
// the caller's stream when an operand of a weight gradient is ready, and on
// the side stream when a weight gradient has read its operands.
enum TrainEvent { kEvDxFc2, kEvDzFc1, kEvDxO, kEvDzQkv, kEvWFc2, kEvWFc1, kEvWO, kEvWQkv,
                  kEvFork, kEvJoin };

// Byte offsets of one block's transposed weights in vl_model::wT.
struct WtOffsets {
  size_t qkv, o, fc1, fc2, per_layer;
};
WtOffsets wt_offsets(const vl_model* m) {
  const size_t D = m->D, F = m->F, es = sizeof(bf16_t);
  WtOffsets w;
  w.qkv = 0;
  w.o = w.qkv + es * 3 * D * D;
  w.fc1 = w.o + es * D * D;
  w.fc2 = w.fc1 + es * D * F;
  w.per_layer = w.fc2 + es * F * D;
  return w;
}

// The backward pass, block by block in reverse.  dX is the gradient of the
// residual stream; every linear layer's input gradient is a GEMM against the
// transposed weight and its weight gradient a GEMM over the tokens (K = T,
// zero-padded to a multiple of 64) of transposed operands; in the BF16 model
// the GEMM operands (dX, dGELU, dQKV and the kept activations) are BF16 and
// the accumulation FP32.  With a side stream (K-major weight gradients), the
// four weight-gradient GEMMs of each block run there, overlapped with the
// input-gradient chain on s; s waits before it overwrites an operand they
// read (dX's BF16 copy, dZ), and the split-K partial buffer is used on the
// side stream only.
vl_status run_backward_body(vl_model* m, const TrainPlan& tp, const float* pix, const float* demb,
                            float* grads, char* ws, hipStream_t s, hipStream_t side) {
  const Part& p = tp.p.parts[0];
  const bool f32 = m->prec == VL_FP32, bf = !f32;
  const ImgDesc* d_imgs = reinterpret_cast<const ImgDesc*>(ws + p.off_imgs);
  const AttnItem* d_items64 = reinterpret_cast<const AttnItem*>(ws + tp.off_items64);
  const AttnItem* d_items128 = reinterpret_cast<const AttnItem*>(ws + tp.off_items128);
  int2* tok = reinterpret_cast<int2*>(ws + p.off_tok);
  const float* X = reinterpret_cast<const float*>(ws + p.off_X);
  void* QH = ws + p.off_QH;
  const int T = p.T, D = m->D, F = m->F, Tp = tp.Tp;
  const float eps = m->cfg.ln_eps;
  float* dX = reinterpret_cast<float*>(ws + tp.dX);
  void* dXb = ws + tp.dXb;
  void* gT = ws + tp.gT;
  void* actT = ws + tp.actT;
  float* dGf = reinterpret_cast<float*>(ws + tp.dGf);
  void* dZ = ws + tp.dZ;
  float* dY = reinterpret_cast<float*>(ws + tp.dY);
  void* Wt = ws + tp.Wt;   // transposed weights of the FP32 path
  const WtOffsets wo = wt_offsets(m);
  float* part = reinterpret_cast<float*>(ws + tp.part);
  float* pg = reinterpret_cast<float*>(ws + tp.pg);
  float* pb = reinterpret_cast<float*>(ws + tp.pb);
  const BlobOffsets bo = blob_offsets(m);
  auto G = [&](size_t off) { return grads + off; };

  VL_HIP(fill_zero(dX, (size_t)T * D, s));
  if (tp.map.on) {
    const vl_status sm = map_head_backward(m, tp, ws, demb, grads, bo, s);
    if (sm != VL_OK) return sm;
  } else {
    VL_HIP(pool_backward(X, d_imgs, p.n, reinterpret_cast<const float*>(ws + p.off_E), demb,
                         m->proj, m->lnf_g, m->lnf_b, eps, D, m->Pd,
                         reinterpret_cast<float*>(ws + tp.de), reinterpret_cast<float*>(ws + tp.zp),
                         dX, reinterpret_cast<float*>(ws + tp.ppg),
                         reinterpret_cast<float*>(ws + tp.ppb), part, G(bo.proj), G(bo.lnf_g),
                         G(bo.lnf_b), s));
  }
  // BF16 models whose widths are multiples of 256 form the weight gradients
  // from the token-major operands (no transposed copies); the passes over
  // the output gradients still run for their column-sum partials (and dX's
  // BF16 copy) but write no transposed matrix.
  const bool km = bf && m->kmajor_wgrad && D % 256 == 0 && F % 256 == 0;
  void* gTo = km ? nullptr : gT;
  const bool ovl = km && side != nullptr;
  hipStream_t sw = ovl ? side : s;   // the weight gradients' stream
  auto rec = [&](int i, hipStream_t st) -> vl_status {
    if (ovl) VL_HIP(hipEventRecord(m->tev[i], st));
    return VL_OK;
  };
  auto wait = [&](hipStream_t st, int i) -> vl_status {
    if (ovl) VL_HIP(hipStreamWaitEvent(st, m->tev[i], 0));
    return VL_OK;
  };
  void* dOb = bf ? static_cast<void*>(ws + tp.dOb) : nullptr;
  // dX in the GEMM operand type (BF16 copy, or dX itself) and transposed; in
  // BF16 models one pass forms the transpose, the copy and the column-sum
  // partials of dX for the bias gradient.
  auto prep_dx = [&]() -> vl_status {
    VL_HIP(transpose_rows(dX, false, T, D, D, gTo, bf, Tp, s, bf ? part : nullptr,
                          bf ? static_cast<bf16_t*>(dXb) : nullptr));
    return VL_OK;
  };
  // Bias gradient = column sums of the layer's output gradient: from the
  // partials its transpose left (BF16), or a pass of its own.
  const int nbc = (T + kColRows - 1) / kColRows;
  auto bias_grad = [&](const void* g, bool g_bf16, int C, float* out) -> vl_status {
    if (bf) VL_HIP(colsum_final(part, nbc, C, out, s));
    else VL_HIP(colsum(g, g_bf16, T, C, C, nullptr, part, out, s));
    return VL_OK;
  };
  for (int l = m->L - 1; l >= 0; --l) {
    const Layer& ly = m->layers[l];
    const TrainLayer& sv = tp.layers[l];
    const BlobOffsets::L& go = bo.layers[l];
    // this block's transposed weights: kept by the model (BF16), or formed
    // here into scratch (FP32)
    const char* wl = bf ? m->wT + wo.per_layer * l : nullptr;
    vl_status st;
    // ---- FC2: x_out = h + GELU(z1) W2^T + b2
    const bool later = l < m->L - 1;   // the previous block's weight gradients may still read
    if (later && (st = wait(s, kEvWO)) != VL_OK) return st;        // ... dX's copy
    if ((st = prep_dx()) != VL_OK) return st;
    if ((st = rec(kEvDxFc2, s)) != VL_OK) return st;
    const void* W2t = bf ? static_cast<const void*>(wl + wo.fc2) : Wt;            // W2^T [F, D]
    if (!bf) VL_HIP(transpose_rows(ly.fc2_w, bf, D, F, F, Wt, bf, D, s));
    if (later && (st = wait(s, kEvWQkv)) != VL_OK) return st;      // ... and dZ
    // g = GELU(z1): kept by the forward (BF16), formed again here (FP32)
    void* g = bf ? static_cast<void*>(ws + sv.g) : QH;
    if (bf) {   // dz1 = (dX W2) GELU'(z1) from the GEMM's epilogue
      EpiArgs eg;
      eg.out = dZ; eg.aux = reinterpret_cast<const float*>(ws + sv.z1); eg.ldo = F;
      VL_HIP(gemm_bf16(static_cast<const bf16_t*>(dXb), D, W2t, D, false, T, F, D, OP_DGELU, -1,
                       eg, s));
    } else {
      if ((st = gemm_into_f32(m, dXb, D, Wt, D, T, F, D, dGf, F, s)) != VL_OK) return st;
      VL_HIP(gelu_backward(dGf, reinterpret_cast<const float*>(ws + sv.z1), dZ, QH, bf,
                           (size_t)T * F, s));                                   // dz1, g
    }
    if ((st = rec(kEvDzFc1, s)) != VL_OK) return st;   // dZ of FC1 ready
    if (km) {
      if ((st = wait(sw, kEvDxFc2)) != VL_OK) return st;
      st = wgrad_gemm_km(tp, ws, dXb, D, g, F, D, F, G(go.fc2_w), sw);
      if (st == VL_OK) st = rec(kEvWFc2, sw);
    } else {
      VL_HIP(transpose_rows(g, bf, T, F, F, actT, bf, Tp, s));                   // g^T
      st = wgrad_gemm(m, tp, ws, gT, actT, D, F, G(go.fc2_w), s);
    }
    if (st != VL_OK) return st;
    if ((st = bias_grad(dX, false, D, G(go.fc2_b))) != VL_OK) return st;
    // ---- FC1: z1 = y2 W1^T + b1
    const void* W1t = bf ? static_cast<const void*>(wl + wo.fc1) : Wt;            // W1^T [D, F]
    if (!bf) VL_HIP(transpose_rows(ly.fc1_w, bf, F, D, D, Wt, bf, F, s));
    if ((st = gemm_into_f32(m, dZ, F, W1t, F, T, D, F, dY, D, s)) != VL_OK) return st;
    VL_HIP(transpose_rows(dZ, bf, T, F, F, gTo, bf, Tp, s, bf ? part : nullptr));
    if (km) {
      if ((st = wait(sw, kEvDzFc1)) != VL_OK) return st;
      st = wgrad_gemm_km(tp, ws, dZ, F, ws + sv.y2, D, F, D, G(go.fc1_w), sw);
      if (st == VL_OK) st = rec(kEvWFc1, sw);
    } else {
      VL_HIP(transpose_rows(ws + sv.y2, bf, T, D, D, actT, bf, Tp, s));
      st = wgrad_gemm(m, tp, ws, gT, actT, F, D, G(go.fc1_w), s);
    }
    if (st != VL_OK) return st;
    if ((st = bias_grad(dZ, bf, F, G(go.fc1_b))) != VL_OK) return st;
    // ---- LN2 (dX += LN2'(h) dY)
    VL_HIP(layernorm_backward(reinterpret_cast<const float*>(ws + sv.h), ly.ln2_g, dY, eps, dX, T,
                              D, pg, pb, G(go.ln2_g), G(go.ln2_b), s));
    // ---- output projection: h = x + O Wo^T + bo
    if ((st = wait(s, kEvWFc2)) != VL_OK) return st;   // FC2's weight gradient read dX's copy
    if ((st = prep_dx()) != VL_OK) return st;
    if ((st = rec(kEvDxO, s)) != VL_OK) return st;
    const void* Wot = bf ? static_cast<const void*>(wl + wo.o) : Wt;              // W_o^T
    if (!bf) VL_HIP(transpose_rows(ly.o_w, bf, D, D, D, Wt, bf, D, s));
    // dO in FP32, and (BF16) its BF16 copy for the attention backward
    if ((st = gemm_into_f32(m, dXb, D, Wot, D, T, D, D, dY, D, s,
                            bf ? static_cast<bf16_t*>(dOb) : nullptr)) != VL_OK)
      return st;
    if (km) {
      if ((st = wait(sw, kEvDxO)) != VL_OK) return st;
      st = wgrad_gemm_km(tp, ws, dXb, D, ws + sv.o, D, D, D, G(go.o_w), sw);
      if (st == VL_OK) st = rec(kEvWO, sw);
    } else {
      VL_HIP(transpose_rows(ws + sv.o, bf, T, D, D, actT, bf, Tp, s));
      st = wgrad_gemm(m, tp, ws, gT, actT, D, D, G(go.o_w), s);
    }
    if (st != VL_OK) return st;
    if ((st = bias_grad(dX, false, D, G(go.o_b))) != VL_OK) return st;
    // ---- attention
    // (BF16: the log-sum-exp the forward kept, and dO also in BF16; FP32:
    // recomputed)
    if ((st = wait(s, kEvWFc1)) != VL_OK) return st;   // FC1's weight gradient read dZ
    VL_HIP(attention_backward(ws + sv.qkv, ws + sv.o, bf, dY, d_imgs, d_items64, tp.n_items64,
                              d_items128, tp.n_items128,
                              m->heads, m->hd, dZ,
                              reinterpret_cast<float*>(ws + (bf ? sv.lse : tp.lse)),
                              reinterpret_cast<float*>(ws + tp.dsum), s, bf,
                              bf ? static_cast<const bf16_t*>(dOb) : nullptr));
    if ((st = rec(kEvDzQkv, s)) != VL_OK) return st;
    // ---- QKV: [q|k|v] = y1 Wqkv^T + bqkv
    const void* Wqt = bf ? static_cast<const void*>(wl + wo.qkv) : Wt;            // [D, 3D]
    if (!bf) VL_HIP(transpose_rows(ly.qkv_w, bf, 3 * D, D, D, Wt, bf, 3 * D, s));
    if ((st = gemm_into_f32(m, dZ, 3 * D, Wqt, 3 * D, T, D, 3 * D, dY, D, s)) != VL_OK) return st;
    VL_HIP(transpose_rows(dZ, bf, T, 3 * D, 3 * D, gTo, bf, Tp, s, bf ? part : nullptr));
    if (km) {
      if ((st = wait(sw, kEvDzQkv)) != VL_OK) return st;
      st = wgrad_gemm_km(tp, ws, dZ, 3 * D, ws + sv.y1, D, 3 * D, D, G(go.qkv_w), sw);
      if (st == VL_OK) st = rec(kEvWQkv, sw);
    } else {
      VL_HIP(transpose_rows(ws + sv.y1, bf, T, D, D, actT, bf, Tp, s));
      st = wgrad_gemm(m, tp, ws, gT, actT, 3 * D, D, G(go.qkv_w), s);
    }
    if (st != VL_OK) return st;
    if ((st = bias_grad(dZ, bf, 3 * D, G(go.qkv_b))) != VL_OK) return st;
    // ---- LN1 (dX += LN1'(x) dY)
    VL_HIP(layernorm_backward(reinterpret_cast<const float*>(ws + sv.xin), ly.ln1_g, dY, eps, dX,
                              T, D, pg, pb, G(go.ln1_g), G(go.ln1_b), s));
  }
  // ---- token embedding: patches (gathered again), class token, positions
  // (after every weight gradient of the side stream: the split-K partials)
  if (ovl) {
    vl_status sj = rec(kEvJoin, side);
    if (sj == VL_OK) sj = wait(s, kEvJoin);
    if (sj != VL_OK) return sj;
  }
  VL_HIP(im2col(pix, d_imgs, p.n, p.max_ntok, m->cfg.channels, m->P, m->Kpad, QH, bf, tok, s));
  VL_HIP(transpose_rows(dX, false, T, D, D, gT, bf, Tp, s));
  VL_HIP(transpose_rows(QH, bf, T, m->Kpad, m->Kpad, actT, bf, Tp, s));
  float* dwf = reinterpret_cast<float*>(ws + tp.dwf);
  {
    const vl_status st = wgrad_gemm(m, tp, ws, gT, actT, D, m->Kpad, dwf, s);
    if (st != VL_OK) return st;
  }
  VL_HIP(colsum(dX, false, T, D, D, tok, part, G(bo.patch_b), s));
  ChanNorm cn{};
  for (int c = 0; c < 4; ++c) {
    cn.mean[c] = c < m->cfg.channels ? m->cfg.chan_mean[c] : 0.f;
    cn.std[c] = c < m->cfg.channels ? m->cfg.chan_std[c] : 1.f;
  }
  VL_HIP(embed_backward(dX, d_imgs, p.n, D, 1 + m->g0 * m->g0, dwf, m->Kpad, G(bo.patch_b), cn,
                        m->Kpe, m->P * m->P, G(bo.pos), G(bo.cls), G(bo.patch_w), s));
  return VL_OK;
}

// BF16 models: make sure the transposed block weights exist (allocated and
// formed on s by the first call; later calls make s wait for that fill).
vl_status ensure_transposed_weights(vl_model* m, hipStream_t s) {
  if (m->wT) {
    VL_HIP(hipStreamWaitEvent(s, m->wT_ev, 0));
    return VL_OK;
  }
  const WtOffsets o = wt_offsets(m);
  const int D = m->D, F = m->F;
  char* p = nullptr;
  hipError_t e = hipMalloc(&p, o.per_layer * m->L);
  if (e != hipSuccess) {
    (void)hipGetLastError();   // leave no stale error for the next launch check
    return hip_fail(e, "hipMalloc(transposed weights)");
  }
  hipEvent_t ev = nullptr;
  e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  for (int l = 0; l < m->L && e == hipSuccess; ++l) {
    const Layer& ly = m->layers[l];
    char* q = p + o.per_layer * l;
    e = transpose_rows(ly.qkv_w, true, 3 * D, D, D, q + o.qkv, true, 3 * D, s);
    if (e == hipSuccess) e = transpose_rows(ly.o_w, true, D, D, D, q + o.o, true, D, s);
    if (e == hipSuccess) e = transpose_rows(ly.fc1_w, true, F, D, D, q + o.fc1, true, F, s);
    if (e == hipSuccess) e = transpose_rows(ly.fc2_w, true, D, F, F, q + o.fc2, true, D, s);
  }
  if (e == hipSuccess) e = hipEventRecord(ev, s);
  if (e != hipSuccess) {
    // nothing enqueued after a failed launch reads p; wait for the rest
    (void)hipStreamSynchronize(s);
    (void)hipFree(p);
    if (ev) (void)hipEventDestroy(ev);
    return hip_fail(e, "transposed weights");
  }
  m->wT = p;
  m->wT_ev = ev;
  return VL_OK;
}

// The backward on the caller's stream s; with K-major weight gradients the
// model's side stream takes them (forked after everything before this call
// on s, joined back into s before returning, also after an error).
vl_status run_backward(vl_model* m, const TrainPlan& tp, const float* pix, const float* demb,
                       float* grads, char* ws, hipStream_t s) {
  const bool km = m->prec == VL_BF16 && m->kmajor_wgrad && m->D % 256 == 0 && m->F % 256 == 0;
  hipStream_t side = nullptr;
  if (m->prec == VL_BF16) {
    const vl_status sw = ensure_transposed_weights(m, s);
    if (sw != VL_OK) return sw;
  }
  if (km) {
    if (!m->side) VL_HIP(hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking));
    for (hipEvent_t& e : m->tev)
      if (!e) VL_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    VL_HIP(hipEventRecord(m->tev[kEvFork], s));
    VL_HIP(hipStreamWaitEvent(m->side, m->tev[kEvFork], 0));
    side = m->side;
  }
  const vl_status st = run_backward_body(m, tp, pix, demb, grads, ws, s, side);
  if (side && hipEventRecord(m->tev[kEvJoin], side) == hipSuccess)
    (void)hipStreamWaitEvent(s, m->tev[kEvJoin], 0);
  return st;
}

vl_status check_train_args(vl_model* m, const float* pix, const void* a, const void* ws,
                           int32_t n, const int32_t* hs, const int32_t* wsz, size_t ws_bytes,
                           TrainPlan* tp) {
  if (!m) return fail(VL_ERR_INVALID_ARG, "model is NULL");
  if (!pix || !a || !ws) return fail(VL_ERR_INVALID_ARG, "NULL pointer argument");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(VL_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (reinterpret_cast<uintptr_t>(pix) % 16 || reinterpret_cast<uintptr_t>(a) % 16)
    return fail(VL_ERR_INVALID_ARG, "pixels and embedding arrays must be 16-byte aligned");
  std::string why;
  if (!make_train_plan(m, n, hs, wsz, tp, &why)) {
    const bool unsup = m->text || (m->prec != VL_FP32 && m->prec != VL_BF16) ||
                       (m->cfg.pool == VL_POOL_MAP && m->hd > 64);
    return fail(unsup ? VL_ERR_UNSUPPORTED : VL_ERR_INVALID_ARG, why);
  }
  if (ws_bytes < tp->total)
    return fail(VL_ERR_WORKSPACE_TOO_SMALL, "workspace has " + std::to_string(ws_bytes) +
                                                " bytes, needs " + std::to_string(tp->total));
  return VL_OK;
}

}  // namespace

extern "C" {

size_t vl_train_workspace_bytes(const vl_model* m, int32_t n, const int32_t* hs,
                                const int32_t* wsz) {
  if (!m) return 0;
  TrainPlan tp;
  std::string why;
  if (!make_train_plan(m, n, hs, wsz, &tp, &why)) return 0;
  return tp.total;
}

vl_status vl_encode_images_train(vl_model* m, const float* pix, const int32_t* hs,
                                 const int32_t* wsz, int32_t n, float* emb, void* ws,
                                 size_t ws_bytes, void* stream) {
  TrainPlan tp;
  vl_status st = check_train_args(m, pix, emb, ws, n, hs, wsz, ws_bytes, &tp);
  if (st != VL_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  std::lock_guard<std::mutex> lk(m->mu);
  m->train_key.clear();
  st = stage_descriptors(m, tp.p, w, s);
  if (st == VL_OK) st = run_train_forward(m, tp, pix, emb, w, s);
  if (st != VL_OK) return st;
  m->train_key = train_key(tp, pix, ws, ws_bytes);
  return mark_use(m, s);
}

vl_status vl_encode_images_backward(vl_model* m, const float* pix, const int32_t* hs,
                                    const int32_t* wsz, int32_t n, const float* d_emb,
                                    float* grads, void* ws, size_t ws_bytes, void* stream) {
  TrainPlan tp;
  vl_status st = check_train_args(m, pix, d_emb, ws, n, hs, wsz, ws_bytes, &tp);
  if (st != VL_OK) return st;
  if (!grads || reinterpret_cast<uintptr_t>(grads) % 16)
    return fail(VL_ERR_INVALID_ARG, "grads must be non-NULL and 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(m->mu);
  if (m->train_key != train_key(tp, pix, ws, ws_bytes))
    return fail(VL_ERR_INVALID_ARG,
                "no matching vl_encode_images_train call (same pixels, shapes and workspace) "
                "precedes this backward pass");
  st = run_backward(m, tp, pix, d_emb, grads, static_cast<char*>(ws), s);
  if (st != VL_OK) return st;
  return mark_use(m, s);
}

}  // extern "C"
