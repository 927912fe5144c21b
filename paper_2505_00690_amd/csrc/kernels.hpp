// Launchers of the gfx950 kernels (host-callable).  All launchers enqueue on
// `s` and return the launch status; shapes are validated by the caller.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch.hpp"
#include "common.hpp"

namespace vl {

// The contractions of the path.  Each has its own kernel instantiation (so
// profiles name them apart) and a fixed epilogue:
//   OP_PATCH  : X[m,n] = acc + (class token ? cls[n] : bias[n]) + pos(m,n)
//   OP_QKV    : out = acc * ws[n] + bias[n]              (BF16 / FP32 out)
//   OP_OPROJ  : resid[m,n] += acc * ws[n] + bias[n]      (FP32)
//   OP_FC1    : out = GELU(acc * ws[n] + bias[n])        (BF16 / FP32 out)
//   OP_FC2    : resid[m,n] += acc * ws[n] + bias[n]      (FP32)
//   OP_LOGITS : out = alpha * acc + beta                 (FP32; BF16 GEMMs
//               without split-K: with out2 also its BF16 copy [M, ldo])
//   OP_FC1_PRE: out = acc * ws[n] + bias[n]              (FP32 out; the FC1
//               pre-activation the training forward keeps for the backward;
//               with out2 also GELU of it in BF16 [M, ldo], as OP_FC1 forms it)
//   OP_DGELU  : the FC2 input gradient through the GELU (BF16 GEMMs): with
//               z = aux[m,n] (the kept FC1 pre-activation, FP32),
//               out = acc * GELU'(z) and, with out2, out2 = GELU(z), both
//               BF16 [M, ldo]
enum GemmOp { OP_PATCH = 0, OP_QKV = 1, OP_OPROJ = 2, OP_FC1 = 3, OP_FC2 = 4, OP_LOGITS = 5,
              OP_FC1_PRE = 6, OP_DGELU = 7 };

struct EpiArgs {
  const float* bias = nullptr;    // [N]
  const float* wscale = nullptr;  // [N] per-output-row weight scale (FP8)
  void* out = nullptr;            // [M, ldo], BF16 or FP32 (e4m3 codes for MXFP8 FC1)
  int ldo = 0;
  uint8_t* out_scale = nullptr;   // MXFP8 FC1 output: E8M0 scales, [ldo/128][M][4]
  int scale_rows = 0;             //   (M of that layout)
  // patch embedding
  const int2* tok_info = nullptr;  // [M]: (image, token index in image)
  const ImgDesc* imgs = nullptr;
  const float* cls = nullptr;      // [D]
  const float* pos = nullptr;      // [1 + g0*g0, D]
  int base_grid = 0;
  float alpha = 1.f, beta = 0.f;
  // LayerNorm folded into the BF16 / e4m3-weight block GEMMs (not MXFP8).
  // Producer (OP_OPROJ, OP_FC2 residual epilogues) with u_out: also writes
  // u = bf16(x * u_gamma[n]) [M, ldo] of the updated residual x, and per row
  // and 32-column group g the group's mean and sum of squared deviations
  // (mean, M2) of x at part_stats[(g * M + m) * 2] (group-major).
  bf16_t* u_out = nullptr;
  const float* u_gamma = nullptr;
  float* part_stats = nullptr;
  // Consumer (OP_QKV, OP_FC1) with row_stats = (mean, rstd) per row of the
  // LayerNorm input: y = rstd (acc * ws[n] - mean c1[n]) + c2[n] replaces
  // acc * ws[n] + bias[n], where c1 = W gamma and c2 = W beta + bias
  // (so y = LN(x) W^T + bias with the A operand u = x * gamma).
  const float* row_stats = nullptr;
  const float* c1 = nullptr;
  const float* c2 = nullptr;
  // Split-K (BF16 GEMM, OP_LOGITS only): with kc > 0 the launch has
  // ceil(K / kc) splits in grid y; split z sums K columns [z kc, z kc + kc)
  // and writes its FP32 partial product at out + z * zstride.
  int kc = 0;
  size_t zstride = 0;
  // Capacity launches (BF16 GEMMs): the grid covers M rows, the live row
  // count is *m_dev (<= M); tiles past it return at once.
  const int32_t* m_dev = nullptr;
  // Second output and auxiliary input (OP_FC1_PRE, OP_DGELU).
  void* out2 = nullptr;
  const float* aux = nullptr;
  // Residual epilogues (OP_OPROJ, OP_FC2; BF16 and FP32 GEMMs): with
  // resid_in the residual is read from resid_in [M, ldo] and the sum written
  // to out, instead of updating out in place.
  const float* resid_in = nullptr;
};

// Tile configurations of the BF16 GEMM.  Every configuration accumulates K
// in the same order (one MFMA per 16 K values, K ascending), so all give
// bitwise identical results and the choice may depend on the batch size.
enum GemmCfg {
  CFG_DL_256x256_W2x4 = 0,
  CFG_DL_256x256_W4x2 = 1,
  CFG_DL_256x256_W2x2 = 2,
  CFG_DL_128x128_W2x2 = 3,
  CFG_DL_256x128_W2x2 = 4,
  CFG_DL_128x256_W2x2 = 5,
  CFG_REG_128x128_W2x2 = 6,
  CFG_DL_192x256_W2x4 = 7,
  CFG_DL3_160x256_W1x8 = 8,
  N_BF16_CFGS = 9,
  // MXFP8 x MXFP8 configurations (gemm_mx).  All accumulate K in the same
  // order (one scaled MFMA per 64 K values, K ascending).
  CFG_MX_160x256_W1x8 = 9,
  CFG_MX_192x256_W2x4 = 10,
  CFG_MX_128x256_W2x4 = 11,
  CFG_MX_128x128_W2x2 = 12,
  N_GEMM_CFGS = 13
};
const char* gemm_cfg_name(int cfg);
inline bool gemm_cfg_is_mx(int cfg) { return cfg >= N_BF16_CFGS && cfg < N_GEMM_CFGS; }
// Configuration used when none is tuned for an operation.
int gemm_cfg_heuristic(int M, int N, int K, bool b_fp8);
int gemm_mx_cfg_heuristic(int M, int N, int K);

// C[M,N] = A[M,K] . B[N,K]^T with BF16 A and BF16 (or e4m3 when b_fp8) B,
// FP32 accumulation, BF16 output for OP_QKV / OP_FC1, FP32 for OP_LOGITS /
// OP_FC1_PRE.  K % 64 == 0, N % 8 == 0.  cfg < 0 selects the heuristic
// configuration.
hipError_t gemm_bf16(const bf16_t* A, int lda, const void* B, int ldb, bool b_fp8,
                     int M, int N, int K, int op, int cfg, const EpiArgs& e, hipStream_t s);

// C = alpha A^T B + beta with K-major BF16 operands A [K, lda] and B [K, ldb]
// (a weight gradient summed over token rows, with neither operand
// transposed first): FP32 output at e.out [M, e.ldo]; split z over K rows
// [z e.kc, (z + 1) e.kc) writes its partial product at e.out + z e.zstride.
// Rows at or past k_valid read as zero.  M % 256 == N % 256 == 0,
// K % 64 == e.kc % 64 == 0, lda >= M, ldb >= N, both multiples of 8.
hipError_t gemm_bf16_kmajor(const bf16_t* A, int lda, const bf16_t* B, int ldb, int M, int N,
                            int K, int k_valid, const EpiArgs& e, hipStream_t s);

// C[M,N] = A[M,K] . B[N,K]^T with both operands MXFP8: e4m3 codes [rows, K]
// and E8M0 scales [K/128][rows][4] (layout in common.hpp), FP32
// accumulation.  OP_QKV writes BF16; OP_FC1 writes MXFP8 codes to e.out and
// scales to e.out_scale (e.scale_rows = M); OP_OPROJ / OP_FC2 add into the
// FP32 residual.  K % 128 == 0, N % 32 == 0.  A cfg that is not an MX
// configuration selects the heuristic one.
hipError_t gemm_mx(const uint8_t* A, const uint8_t* SA, const uint8_t* B, const uint8_t* SB,
                   int M, int N, int K, int op, int cfg, const EpiArgs& e, hipStream_t s);

// The same contraction in FP32 (FMA), output FP32.  K % 16 == 0, N % 4 == 0.
hipError_t gemm_f32(const float* A, int lda, const float* B, int ldb, int M, int N,
                    int K, int op, const EpiArgs& e, hipStream_t s);

// The same contraction for products whose A has few rows (M of a batch of
// pooled rows or images): K % 4 == 0, N % 4 == 0, lda and ldb multiples of
// 4; not OP_PATCH.  Each output's summation order is independent of M.
hipError_t gemm_f32_rows(const float* A, int lda, const float* B, int ldb, int M, int N,
                         int K, int op, const EpiArgs& e, hipStream_t s);

// LayerNorm of FP32 rows [M, D] -> BF16 or FP32 rows (with bc: rows
// [0, bc->T) of a grid sized for M).
hipError_t layernorm_rows(const float* x, const float* g, const float* b, float eps,
                          void* y, bool y_bf16, int M, int D, hipStream_t s,
                          const BatchCounts* bc = nullptr);

// LayerNorm folding (see EpiArgs): for the first block, u = bf16(x * g) and
// row_stats (mean, rstd) of x [M, D] directly; elsewhere row_stats from the
// (mean, M2) partials of D/32 column groups a residual epilogue wrote.
hipError_t ln_fold_rows(const float* x, const float* g, float eps, bf16_t* u, float* row_stats,
                        int M, int D, hipStream_t s);
hipError_t ln_stats_from_parts(const float* parts, int M, int D, float eps, float* row_stats,
                               hipStream_t s);
// c1[n] = sum_k g[k] W[n,k] and c2[n] = sum_k b[k] W[n,k] + bias[n] for the
// weights as the GEMM uses them (BF16, or e4m3 codes times the row scale).
hipError_t ln_fold_consts(const void* w, bool w_fp8, const float* wscale, const float* g,
                          const float* b, const float* bias, int N, int K, float* c1, float* c2,
                          hipStream_t s);

// LayerNorm of FP32 rows [M, D] -> MXFP8 codes [M, D] + scales [D/128][M][4].
hipError_t layernorm_rows_mx(const float* x, const float* g, const float* b, float eps,
                             uint8_t* codes, uint8_t* scales, int M, int D, hipStream_t s);

// Patch gathering: token rows [T, Kpad] of raw pixels in (c, a, b) order
// over `chans` input planes (class-token rows and the K padding are zero)
// plus tok_info [T].  With bc: images [0, bc->n) of bc->pix.
hipError_t im2col(const float* pix, const ImgDesc* imgs, int n_imgs, int max_ntok, int chans,
                  int patch, int kpad, void* out, bool out_bf16, int2* tok_info,
                  hipStream_t s, const BatchCounts* bc = nullptr);

// Multi-head self-attention over a packed QKV buffer [T, 3D] -> O [T, D],
// within each descriptor's token range; causal: token i attends to 0..i.
// With bc: items [0, bc->n_items) of a grid sized for n_items.  With
// lse_out [T, heads]: each query's log-sum-exp of its scaled scores in log2
// units (max + log2 sum 2^(s - max)), which the training backward reuses.
hipError_t attention_bf16(const bf16_t* qkv, bf16_t* o, const ImgDesc* imgs,
                          const AttnItem* items, int n_items, int heads, int head_dim,
                          bool causal, hipStream_t s, const BatchCounts* bc = nullptr,
                          float* lse_out = nullptr);
// The same with an MXFP8 output: codes [T, D] + scales [D/128][T][4].
hipError_t attention_bf16_mx(const bf16_t* qkv, uint8_t* codes, uint8_t* scales, int T,
                             const ImgDesc* imgs, const AttnItem* items, int n_items,
                             int heads, int head_dim, bool causal, hipStream_t s);
// K/V-resident form for images of 129 .. 640 tokens at head width 64: one
// workgroup per (image, head) over res_imgs[0 .. n_res) (image indices);
// max_tiles = the largest ceil(tokens / 64) among them (<= 10).  Output as
// attention_bf16 (mx = false) or attention_bf16_mx (mx = true), bitwise.
// With bc: images [0, bc->n_res) of a grid sized for n_res.
hipError_t attention_bf16_resident(const bf16_t* qkv, void* out, uint8_t* out_scale, bool mx,
                                   int T, const ImgDesc* imgs, const int* res_imgs, int n_res,
                                   int max_tiles, int heads, int head_dim, hipStream_t s,
                                   const BatchCounts* bc = nullptr, float* lse_out = nullptr);
hipError_t attention_f32(const float* qkv, float* o, const ImgDesc* imgs,
                         const AttnItem* items, int n_items, int heads, int head_dim,
                         bool causal, hipStream_t s);

// Pooling of each sequence's first (class token) or last (pool_last: the
// text end-of-text token) row, final LayerNorm into z [n, D] (scratch),
// projection [P, D] into e_tmp [n, P], then L2 normalisation into emb [n, P].
// D % 4 == 0, P % 4 == 0.  With bc: sequences [0, bc->n) of grids sized for
// n_imgs, written to bc->emb (emb unused).
hipError_t pool_project(const float* x, const ImgDesc* imgs, int n_imgs, const float* g,
                        const float* b, float eps, const float* proj, int D, int P,
                        bool pool_last, float* z, float* e_tmp, float* emb, hipStream_t s,
                        const BatchCounts* bc = nullptr);

// Row-wise division of e [rows, P] by its L2 norm (clamped at 1e-12).
hipError_t l2_normalise_rows(const float* e, float* out, int rows, int P, hipStream_t s);

// Attention pooling with one query per head (MAP head): out [n, D] FP32 from
// the query q [D] and kv [T, 2D] (K | V; BF16 when kv_bf16, else FP32) over
// each image's tokens.  head_dim <= 64 and divides 256.
hipError_t map_attention(const void* kv, bool kv_bf16, const float* q, const ImgDesc* imgs,
                         int n_imgs, int heads, int head_dim, float* out, hipStream_t s);

// Token embedding of packed text sequences (descriptors: tok_start, ntok):
// X [T, D] = tok_emb[id] + pos[index in sequence], and tok_info [T].
hipError_t text_embed(const int32_t* ids, const ImgDesc* seqs, int n_seqs, int max_len,
                      const float* tok_emb, const float* pos, int vocab, int D, float* X,
                      int2* tok_info, hipStream_t s);

// Per-row softmax / sigmoid of logits in place, and the row argmax.
hipError_t score_rows(float* scores, int32_t* top1, int rows, int cols, int head,
                      hipStream_t s);

// Contrastive loss of n matched pairs (head 0 softmax, 1 sigmoid) with its
// gradients: loss[1], dE/dT [n, dim], dsb = (dL/dscale, dL/dbias).  dim %
// 16 == 0; ws holds contrastive_workspace_bytes(n, dim).
size_t contrastive_workspace_bytes(int n, int dim);
// Size of the per-device scratch array of the allocation-free contrastive
// entry point, and its device address on the current device (looked up on
// the first call per device; never allocates).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
hipError_t noalloc_scratch(void** out);
hipError_t contrastive_loss(const float* E, const float* T, int n, int dim, int head,
                            float scale, float bias, float* loss, float* dE, float* dT,
                            float* dsb, void* ws, hipStream_t s);

// ---- training (contrastive training through the image tower)
constexpr int kColRows = 64;   // rows per partial sum of colsum
constexpr int kLnRows = 32;    // rows per partial sum of layernorm_backward
struct ChanNorm { float mean[4], std[4]; };  // per-plane pixel normalisation

// out[c][r] = in[r][c] (rows < rows), zero for rows <= r < ld_out; element
// types BF16 or FP32 (BF16 -> FP32 is not offered).
// With colsum_part (BF16 output, cols % 8 == 0): also the row-block partials
// of colsum for the same input, [ceil(rows / kColRows), cols]; finish with
// colsum_final.  With copy_bf16 (FP32 input, BF16 output): also the input
// rounded to BF16 in its own layout [rows, ld_in].  out may be NULL (BF16
// output type) when colsum_part or copy_bf16 is given: those alone.
hipError_t transpose_rows(const void* in, bool in_bf16, int rows, int cols, int ld_in, void* out,
                          bool out_bf16, int ld_out, hipStream_t s,
                          float* colsum_part = nullptr, bf16_t* copy_bf16 = nullptr);
hipError_t colsum_final(const float* part, int nb, int C, float* out, hipStream_t s);
// out[c] = sum over rows of in[r][c] (class-token rows skipped when tok is
// given), via part [ceil(R / kColRows), C] in a fixed order.  C % 4 == 0,
// ld % 4 == 0.
hipError_t colsum(const void* in, bool in_bf16, int R, int C, int ld, const int2* tok,
                  float* part, float* out, hipStream_t s);
// dx += LayerNorm backward of rows [R, D]; dgamma, dbeta (overwritten) via
// partials pg, pb [ceil(R / kLnRows), D].
hipError_t layernorm_backward(const float* x, const float* g, const float* dy, float eps,
                              float* dx, int R, int D, float* pg, float* pb, float* dgamma,
                              float* dbeta, hipStream_t s);
// g = GELU(z) as the FC1 epilogue forms it (n even); backward dz = dg GELU'(z)
// with g formed again.
hipError_t gelu_forward(const float* z, void* g, bool g_bf16, size_t n, hipStream_t s);
hipError_t gelu_backward(const float* dg, const float* z, void* dz, void* g, bool bf16, size_t n,
                         hipStream_t s);
// dQKV [T, 3D] of the attention of every image: items64 are (image, first
// token) blocks of 64 tokens (FP32 kernels), items128 blocks of 128 tokens
// (BF16 kernels); lse and dsum [T, heads] are scratch, except
// that with lse_given (BF16) lse already holds the forward's log-sum-exp
// (attention_bf16's lse_out) and is only read.  BF16 models also pass dO
// rounded to BF16 (dO_bf16 [T, D]), from which the dK/dV pass loads its tiles.
hipError_t attention_backward(const void* qkv, const void* o, bool bf16, const float* dO,
                              const ImgDesc* imgs, const AttnItem* items64, int n_items,
                              const AttnItem* items128, int n_items128, int heads, int head_dim,
                              void* dqkv, float* lse, float* dsum, hipStream_t s,
                              bool lse_given = false, const bf16_t* dO_bf16 = nullptr);
// Pooling head: de, z [n, *] scratch, the class rows of dX, and the
// gradients of the projection and the final LayerNorm (pg, pb [n, D] and
// part [ceil(n / kColRows), D] scratch).
hipError_t pool_backward(const float* X, const ImgDesc* imgs, int n, const float* e,
                         const float* demb, const float* proj, const float* g, const float* b,
                         float eps, int D, int P, float* de, float* z, float* dX, float* pg,
                         float* pb, float* part, float* d_proj, float* d_lnf_g, float* d_lnf_b,
                         hipStream_t s);
// Position table / class token (images at the base grid) and the unfolded
// patch weights from the folded weights' gradient dwf [D, kpad].
hipError_t embed_backward(const float* dX, const ImgDesc* imgs, int n, int D, int rows_pos,
                          const float* dwf, int kpad, const float* db, ChanNorm cn, int kpe,
                          int pp, float* d_pos, float* d_cls, float* d_patch_w, hipStream_t s);
// out [P, D] = sum over rows i (ascending) of a[i] (x) b[i], a [n, P], b [n, D].
hipError_t outer_sum(const float* a, const float* b, int n, int P, int D, float* out,
                     hipStream_t s);
// Attention-pooling head backward pieces: the L2 normalisation and
// projection of the pooled rows (de [n, P], dz = W_p^T de [n, D]; P <= 1024),
// and the one-query attention per (image, head) (dkv [T, 2D] = [dK | dV] in
// kv's element type, dq [n, D]; head_dim <= 64, images of <= 4096 tokens).
hipError_t l2proj_backward(const float* e, const float* demb, const float* proj, int n, int D,
                           int P, float* de, float* dz, hipStream_t s);
hipError_t map_attention_backward(const void* kv, bool kv_bf16, const float* q, const float* o,
                                  const float* dO, const ImgDesc* imgs, int n, int max_ntok,
                                  int heads, int hd, void* dkv, float* dq, hipStream_t s);
hipError_t fill_zero(float* p, size_t n, hipStream_t s);
// out[i] = sum over z = 0 .. splits-1 (ascending) of part[z * n + i].
hipError_t sum_splits(const float* part, int splits, size_t n, float* out, hipStream_t s);

// FP32 -> BF16 rounding as the kernels do it (method 0: integer RNE of the
// bit pattern; 1: the packed conversion instruction).  n even.
hipError_t bf16_round(const float* src, bf16_t* dst, size_t n, int method, hipStream_t s);

// Weight preparation.
hipError_t convert_bf16(const float* src, bf16_t* dst, size_t n, hipStream_t s);
hipError_t quantise_e4m3_rows(const float* src, uint8_t* dst, float* scales, int rows,
                              int cols, hipStream_t s);
// MXFP8 encoding of FP32 rows [rows, cols] (cols % 128 == 0): codes
// [rows, cols] and scales [cols/128][rows][4].
hipError_t mx_quantise_rows(const float* src, uint8_t* codes, uint8_t* scales, int rows,
                            int cols, hipStream_t s);
hipError_t fold_patch_weights(const float* w, const float* b, const float* mean,
                              const float* stdv, int chans, int D, int patch, int kpad,
                              float* w_f32, bf16_t* w_bf16, float* b_out, hipStream_t s);
hipError_t copy_f32(const float* src, float* dst, size_t n, hipStream_t s);

}  // namespace vl
