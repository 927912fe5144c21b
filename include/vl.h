/*
 * vl.h -- C ABI of the MI355X (gfx950) contrastive image-encoder library.
 *
 * The library computes, entirely in hand-written HIP kernels:
 *   vl_encode_images : pixels -> unit image embeddings.  A ViT image tower
 *       (Dosovitskiy et al., ICLR 2021, Sec. 3.1, Eq. 1-4): per-channel
 *       normalisation, P x P patch embedding, class token, (bilinearly
 *       resampled, Sec. 3.2) position embedding, L pre-LN blocks of
 *       multi-head self-attention (Vaswani et al. 2017, Sec. 3.2, Eq. 1) and
 *       a GELU MLP (Hendrycks & Gimpel 2016), final LayerNorm on the class
 *       token, bias-free projection and L2 normalisation (CLIP, Radford et
 *       al. 2021, Sec. 2.3).
 *   vl_score : logits l_ij = scale * <e_i, t_j> + bias against resident text
 *       embeddings, then a softmax over texts per image (CLIP, Sec. 3.1.2) or
 *       a sigmoid per pair (SigLIP, Zhai et al. 2023, Eq. 1), plus top-1.
 * The URBAN-SIM paper (arXiv 2505.00690) consumes per-environment RGB-D
 * frames at 128x128 in its navigation policy (Appendix, navigation
 * benchmark, observation spaces); it does not itself specify an encoder.
 *
 * Conventions
 *  - Every pointer named *_dev is device memory on the current HIP device and
 *    is owned by the caller; the library never frees it.  Host arrays are
 *    read during the call only.
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream) and never synchronises the device.  Outputs are valid once the
 *    stream reaches the call.
 *  - Arguments are validated before anything is enqueued.  On any error
 *    nothing is enqueued, outputs are untouched, and vl_last_error_message()
 *    returns a description (thread-local).  A HIP failure after enqueue
 *    returns VL_ERR_DEVICE.
 *  - A model may be used from several host threads on different streams,
 *    provided each concurrent call has its own workspace.
 */
#ifndef VL_H_
#define VL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VL_ABI_VERSION 2

typedef enum vl_status {
  VL_OK = 0,
  VL_ERR_INVALID_ARG = 1,
  VL_ERR_UNSUPPORTED = 2,
  VL_ERR_WORKSPACE_TOO_SMALL = 3,
  VL_ERR_DEVICE = 4,
  VL_ERR_INTERNAL = 5
} vl_status;

/* Arithmetic of the encoder.
 *  VL_FP32       : every operand and accumulator FP32.
 *  VL_BF16       : block linear weights rounded to BF16 (round to nearest
 *                  even); GEMM and attention operands BF16 with FP32
 *                  accumulation; residual stream, LayerNorm statistics,
 *                  softmax max/sum, final LayerNorm, projection and L2 norm
 *                  FP32.
 *  VL_FP8W_BF16A : as VL_BF16, but the four per-block linear weights (QKV,
 *                  output projection, FC1, FC2) are OCP e4m3fn codes with one
 *                  FP32 scale per output row, s_o = max_k |W_ok| / 448,
 *                  q = sat(RNE(W / s_o)) (OFP8 rev 1.0, Sec. 5.1).  Codes are
 *                  widened to BF16 exactly inside the GEMM and the scale is
 *                  applied to the FP32 accumulator.
 *  VL_MXFP8      : as VL_BF16, but both operands of the four per-block
 *                  linear layers are MXFP8 (OCP Microscaling Formats (MX)
 *                  Specification v1.0, E4M3 elements with an E8M0 scale per
 *                  block, and its FP32-to-MX conversion rule): every 32 consecutive values
 *                  along the contraction share one power-of-two scale 2^X,
 *                  X = max(floor(log2 max|v|) - 8, -127), and are stored as
 *                  sat448(RNE_e4m3(v / 2^X)).  The weights are encoded once
 *                  at model creation; the activations (both LayerNorm
 *                  outputs, the attention output and the GELU output) are
 *                  encoded by the kernels that produce them, from their
 *                  FP32 values.  The GEMMs multiply codes with the gfx950
 *                  scaled FP8 MFMA, which applies the scales in hardware,
 *                  and accumulate in FP32.  The patch embedding, attention
 *                  (BF16 Q/K/V) and everything else are as in VL_BF16.      */
typedef enum vl_precision {
  VL_FP32 = 0,
  VL_BF16 = 1,
  VL_FP8W_BF16A = 2,
  VL_MXFP8 = 3
} vl_precision;

typedef enum vl_head {
  VL_HEAD_SOFTMAX = 0, /* p_ij = softmax_j(l_ij)          */
  VL_HEAD_SIGMOID = 1  /* p_ij = 1 / (1 + exp(-l_ij))     */
} vl_head;

/* Model dimensions.  width % heads == 0 and head_dim = width/heads must be
 * 32 or 64; width % 128 == 0; mlp % 128 == 0; proj_dim % 4 == 0;
 * width <= 1024.  ln_eps is the LayerNorm epsilon (biased variance).
 * channels: input planes per pixel, 1..4 (3 for RGB; 4 for the RGB-D
 * observations of the paper's navigation benchmark, Appendix, observation
 * spaces).  Pixels are normalised as (x - chan_mean[c]) / chan_std[c] for
 * c < channels (entries past `channels` are ignored).                      */
typedef struct vl_config {
  int32_t patch;
  int32_t width;
  int32_t layers;
  int32_t heads;
  int32_t mlp;
  int32_t proj_dim;
  int32_t base_grid; /* the position table covers base_grid x base_grid  */
  float ln_eps;
  float chan_mean[4];
  float chan_std[4];
  int32_t channels;
  int32_t pool;      /* vl_pool                                            */
} vl_config;

/* Pooling of the final token states into one vector per image.
 *  VL_POOL_CLS : final LayerNorm of the class token (ViT Eq. 4, CLIP).
 *  VL_POOL_MAP : multi-head attention pooling with a learned query (the
 *                SigLIP image tower's head; pooling by multihead attention,
 *                Lee et al. 2019, Set Transformer, Sec. 3.2): the final
 *                LayerNorm on every token, then one attention of the learned
 *                probe (projected by its own Q weights) over the image's
 *                tokens (own K/V projections, `heads` heads), the output
 *                projection, then x + MLP(LN(x)) with GELU and width `mlp`.
 *                The K/V projection runs as a BF16 GEMM in every precision
 *                but VL_FP32; the rest of the head is FP32.
 * Either is followed by the bias-free projection and L2 normalisation.    */
typedef enum vl_pool { VL_POOL_CLS = 0, VL_POOL_MAP = 1 } vl_pool;

typedef struct vl_model vl_model; /* opaque; immutable after creation */

/* Number of FP32 values in the weight blob for `cfg`, 0 if cfg is invalid.
 * Blob layout: tensors back to back, each C-contiguous, in this order
 *   patch_w [D,C,P,P]  patch_b [D]  cls [D]  pos [1+g0*g0, D]   (C = channels)
 *   for each of the L blocks:
 *     ln1_g [D] ln1_b [D] qkv_w [3D,D] qkv_b [3D] o_w [D,D] o_b [D]
 *     ln2_g [D] ln2_b [D] fc1_w [F,D] fc1_b [F] fc2_w [D,F] fc2_b [D]
 *   lnf_g [D]  lnf_b [D]
 *   with VL_POOL_MAP only: probe [D]  q_w [D,D] q_b [D]  kv_w [2D,D]
 *     kv_b [2D] (rows [K | V])  o_w [D,D] o_b [D]  ln_g [D] ln_b [D]
 *     fc1_w [F,D] fc1_b [F]  fc2_w [D,F] fc2_b [D]
 *   proj_w [P_dim, D]
 * Linear weights are [out, in] (y = x W^T + b).  qkv_w's rows are
 * [Q | K | V]; head k uses rows/columns k*d .. k*d+d-1 of each part.  The
 * position table's row 0 belongs to the class token; rows 1.. are the
 * g0 x g0 grid, row-major.                                                  */
size_t vl_weights_count(const vl_config* cfg);

/* Build a model from an FP32 weight blob (device, caller-owned, may be freed
 * once the stream has passed this call).  The library allocates its own
 * device copy of the weights in the requested precision (hipMalloc), folds
 * the pixel normalisation into the patch embedding, and enqueues the
 * conversion kernels on `stream`.  *out receives the handle.
 * Errors: VL_ERR_INVALID_ARG (null pointers, bad dims, n_floats mismatch),
 * VL_ERR_UNSUPPORTED (head_dim not 32/64, width > 1024), VL_ERR_DEVICE.    */
vl_status vl_model_create(const vl_config* cfg, vl_precision prec,
                          const float* weights_dev, size_t n_floats,
                          void* stream, vl_model** out);

/* Frees the model's device memory and cached graphs.  First waits for the
 * model's own enqueued work to finish: every call records an event on the
 * stream it ran on (and creation on its stream), and destroy waits for the
 * latest event of each such stream and for the model's internal stream; it
 * does not synchronise the device.  NULL ok.                              */
void vl_model_destroy(vl_model* m);

/* ---- Text tower ---------------------------------------------------------
 * The text encoder of a contrastive model (CLIP, Radford et al. 2021,
 * Sec. 2.4): token embedding plus a learned absolute position embedding, L
 * pre-LN blocks identical to the image tower's except that self-attention
 * is causal (token i attends to tokens 0..i of its own sequence), then the
 * final LayerNorm of the sequence's last token (its end-of-text token),
 * the bias-free projection and L2 normalisation.  The embeddings it returns
 * are the `texts` operand of vl_score.                                      */
typedef struct vl_text_config {
  int32_t vocab;     /* token table rows                                    */
  int32_t ctx;       /* longest sequence (position table rows), <= 1024     */
  int32_t width;     /* width % 128 == 0, head_dim 32 or 64, width <= 1024  */
  int32_t layers;
  int32_t heads;
  int32_t mlp;       /* mlp % 128 == 0                                      */
  int32_t proj_dim;  /* % 4 == 0, <= 1024                                   */
  float ln_eps;
} vl_text_config;

/* FP32 values in a text model's weight blob, 0 if cfg is invalid.  Layout,
 * tensors back to back, C-contiguous:
 *   tok_emb [vocab, D]  pos [ctx, D]
 *   per block: as for images (ln1_g .. fc2_b)
 *   lnf_g [D]  lnf_b [D]  proj_w [P_dim, D]                                */
size_t vl_text_weights_count(const vl_text_config* cfg);

/* Build a text model; arguments, precisions and errors as vl_model_create.
 * The handle works with vl_model_destroy, vl_model_set_option and
 * vl_model_op_times (operation 0 is then the token embedding); GEMM tiles
 * use the built-in heuristic or vl_model_set_tuning (the autotuner takes
 * images only).                                                             */
vl_status vl_text_model_create(const vl_text_config* cfg, vl_precision prec,
                               const float* weights_dev, size_t n_floats,
                               void* stream, vl_model** out);

/* Workspace bytes for vl_encode_texts of n_texts sequences of the given
 * lengths (host array); 0 on invalid input or a non-text model.           */
size_t vl_text_workspace_bytes(const vl_model* m, int32_t n_texts,
                               const int32_t* lengths);

/* Encode n_texts token sequences.
 *  ids_dev     : int32 token ids of all sequences back to back (sequence i
 *                has lengths[i] ids, 1 <= lengths[i] <= ctx, ending with its
 *                end-of-text token), 4-byte aligned.  Ids outside
 *                [0, vocab) are clamped into it (never read out of bounds).
 *  lengths     : host array of n_texts lengths (1 <= n_texts <= 65535).
 *  emb_out_dev : [n_texts, proj_dim] FP32 unit rows, 16-byte aligned.
 *  workspace_dev : >= vl_text_workspace_bytes(...), 256-byte aligned.
 * Sequences are packed into one token stream; attention never crosses
 * sequences.                                                                */
vl_status vl_encode_texts(vl_model* m, const int32_t* ids_dev, const int32_t* lengths,
                          int32_t n_texts, float* emb_out_dev, void* workspace_dev,
                          size_t workspace_bytes, void* stream);

/* Options (all off by default).  Setting an option waits only for the
 * cached graphs it drops (each graph's last replay); it does not synchronise
 * the device.
 *   VL_OPT_GRAPHS : 1 = capture calls into HIP graphs on first use and
 *                   replay them.  For VL_BF16 and VL_FP8W_BF16A image models
 *                   with VL_POOL_CLS and VL_OPT_FUSED_LN off, a graph serves
 *                   a capacity bucket: each part's token count is rounded
 *                   up (counts <= 16 exact; above, to a multiple of a
 *                   quarter of the power of two below, never reaching the
 *                   next power of two) and its image count to a power of
 *                   two; kernel grids are sized for the
 *                   capacities, and the kernels read the call's counts,
 *                   descriptors, pixel and output pointers from the
 *                   workspace, uploaded ahead of the replay on the call's
 *                   stream.  So different batches of one bucket (other
 *                   image sizes, pixel and output buffers) replay one graph
 *                   for a workspace and stream, with the same bits as an
 *                   eager call.  vl_encode_workspace_bytes then returns the
 *                   bucket's size (up to ~1/4 more), so query it after
 *                   setting this option.  Other models key a graph on the
 *                   exact call (shapes, pointers, stream).  At most 256
 *                   graphs are kept per model; the least recently replayed
 *                   one is dropped (after its last replay finishes) to make
 *                   room.
 *   VL_OPT_TIMING : 1 = bracket every kernel launch of vl_encode_images
 *                   with HIP events on the stream it runs on and accumulate
 *                   per-operation device time (read with
 *                   vl_model_op_times).  Calls made while timing is on are
 *                   launched eagerly even if VL_OPT_GRAPHS is set.
 *   VL_OPT_SPLIT  : 1 = run a BF16, FP8-weight or MXFP8 batch of at least 4096
 *                   tokens as two parts of consecutive images (about half
 *                   the tokens each); the second part runs on a stream the
 *                   library owns, forked from and joined back into the
 *                   call's stream, so the parts overlap.  Outputs are
 *                   bitwise identical to a one-part run.  0 = one part on
 *                   the call's stream.  Changing it drops cached graphs.
 *                   The training forward (vl_encode_images_train, VL_BF16)
 *                   splits the same way.  (On MI355X at ViT-L/14@336, batch
 *                   32, two parts run 6-7 % faster than one.)
 *   VL_OPT_FUSED_LN : off by default (VL_BF16 and VL_FP8W_BF16A; no effect
 *                   on other precisions).  Both LayerNorms of a block are
 *                   folded into the GEMMs around them: the residual
 *                   epilogues of the output projection and FC2 also write
 *                   u = bf16(x * gamma) of the next LayerNorm and per-row
 *                   partial statistics (mean and sum of squared deviations
 *                   of each 32-column group, FP32); a small pass combines
 *                   them into the row's mean and 1/sqrt(var + eps); QKV and
 *                   FC1 multiply u by the weights and form
 *                   rstd (acc - mean W gamma) + W beta + bias in their
 *                   epilogues.  The same function as LayerNorm then linear
 *                   layer; the BF16 operand is x * gamma instead of the
 *                   normalised row, so results differ from 0 by rounding.
 *                   (Measured on MI355X at ViT-L/14@336, batch 32: the
 *                   LayerNorm time falls but the four GEMMs lose more, ~5 %
 *                   slower per step, hence off.)  Changing it drops cached
 *                   graphs.
 *   VL_OPT_ATTN_RESIDENT : on by default (BF16 attention at head width 64,
 *                   image towers).  Images of 129 .. 640 tokens run their
 *                   attention with one workgroup per (image, head) that
 *                   loads the head's keys and values into LDS once and
 *                   serves every query of the image from them; other images
 *                   stream key / value tiles per block of 128 queries.  Both
 *                   forms give the same bits.  Changing it drops cached
 *                   graphs.
 *   VL_OPT_GRAPH_BUCKETS : on by default.  0 = key every graph on the exact
 *                   call, also for the models that would plan capacity
 *                   buckets (a fixed-shape workload then launches grids of
 *                   exactly its size).  Changing it drops cached graphs and
 *                   changes what vl_encode_workspace_bytes returns.
 *   VL_OPT_KMAJOR_WGRAD : on by default (VL_BF16 training with width and MLP
 *                   width multiples of 256).  The weight gradients of the
 *                   encoder blocks read the token-major output gradients
 *                   and activations directly; 0 = transpose both into
 *                   scratch first.  Same operands and splits: results
 *                   differ only in FP32 summation order.                   */
typedef enum vl_option { VL_OPT_GRAPHS = 0, VL_OPT_TIMING = 1, VL_OPT_SPLIT = 2,
                         VL_OPT_FUSED_LN = 3, VL_OPT_ATTN_RESIDENT = 4,
                         VL_OPT_GRAPH_BUCKETS = 5, VL_OPT_KMAJOR_WGRAD = 6 } vl_option;
vl_status vl_model_set_option(vl_model* m, vl_option opt, int64_t value);

/* Operations of the encoder, as reported by vl_model_op_times:
 *   0 patch embedding (patch gather + GEMM with bias/class/position add)
 *   1 LayerNorm (both per block)      2 QKV GEMM          3 attention
 *   4 output projection GEMM (+ residual)                 5 FC1 GEMM (+ GELU)
 *   6 FC2 GEMM (+ residual)           7 pooling, final LayerNorm, projection,
 *                                       L2 normalisation                   */
#define VL_N_OPS 8

/* Waits for all timed launches recorded so far, then writes the summed
 * device milliseconds and the launch count of each operation into
 * ms_out[VL_N_OPS] and launches_out[VL_N_OPS] (host arrays; either may be
 * NULL).  reset != 0 clears the totals afterwards.                         */
vl_status vl_model_op_times(vl_model* m, double* ms_out, int64_t* launches_out,
                            int32_t reset);

/* Graph cache counters since the model was created: graphs captured,
 * replays (a captured graph's first launch counts as a replay), graphs
 * held now.  Any pointer may be NULL.  Host-only.                          */
vl_status vl_model_graph_stats(vl_model* m, int64_t* captures, int64_t* replays,
                               int32_t* cached);

/* ---- GEMM tile configurations and the autotuner ------------------------
 * The BF16 / e4m3-weight GEMMs (patch embedding, QKV, output projection,
 * FC1, FC2) can run in several tile configurations.  All of them accumulate
 * K in the same order, so they give bitwise identical results: the choice
 * only affects speed, and may differ with the batch size.  The choice is a
 * table indexed by (GEMM operation, M bucket), where M is the packed token
 * count of the call and the bucket is floor(log2(M)); -1 entries use the
 * built-in heuristic.  Not used by VL_FP32 models.                        */
#define VL_N_GEMM_OPS 5       /* 0 patch, 1 qkv, 2 oproj, 3 fc1, 4 fc2      */
#define VL_N_M_BUCKETS 25

int32_t vl_gemm_config_count(void);
/* Name of configuration `cfg` (static string), NULL if out of range.      */
const char* vl_gemm_config_name(int32_t cfg);

/* Copy the model's table (VL_N_GEMM_OPS * VL_N_M_BUCKETS int32, row-major
 * by operation) to / from host memory.  set validates every entry (-1 or a
 * valid id) and drops cached graphs.                                       */
vl_status vl_model_get_tuning(const vl_model* m, int32_t* table);
vl_status vl_model_set_tuning(vl_model* m, const int32_t* table);

/* Persist the tuning table as JSON (path: a file the call writes / reads):
 *   {"abi": 2, "arch": "gfx950", "precision": "bf16", "text": false,
 *    "width": D, "mlp": F, "patch_k": padded patch length,
 *    "table": {"qkv_gemm": {"<M bucket>": "<configuration name>", ...}, ...}}
 * Only tuned entries are written.  load validates the file against the
 * model (ABI, device architecture, precision, image or text model, GEMM
 * dimensions) and every name, then applies it as vl_model_set_tuning does;
 * on any mismatch it returns VL_ERR_INVALID_ARG and leaves the table as it
 * was.  Host-only calls (no device work).                                  */
vl_status vl_model_save_tuning(const vl_model* m, const char* path);
vl_status vl_model_load_tuning(vl_model* m, const char* path);

/* Autotune for one batch shape: runs one full vl_encode_images of the given
 * batch (so the workspace holds live operands), then times every
 * configuration of each GEMM operation over `reps` launches with HIP events
 * on `stream`, and stores the fastest for this batch's M bucket.  When every
 * part of the batch falls in one M bucket, the choice for each block GEMM
 * among the configurations within 5 % of its fastest is then made by timing
 * `reps` whole encoder passes per candidate.  Arguments
 * as for vl_encode_images; emb_out_dev receives that encode's result.
 * Blocks until the timing is done.  VL_ERR_UNSUPPORTED for VL_FP32.       */
vl_status vl_model_autotune(vl_model* m, const float* pixels_dev, const int32_t* heights,
                            const int32_t* widths, int32_t n_images, float* emb_out_dev,
                            void* workspace_dev, size_t workspace_bytes, int32_t reps,
                            void* stream);

/* Bytes of device workspace vl_encode_images needs for this batch.
 * heights/widths: host arrays of n_images entries.  0 on invalid input.   */
size_t vl_encode_workspace_bytes(const vl_model* m, int32_t n_images,
                                 const int32_t* heights, const int32_t* widths);

/* Encode n_images images.
 *  pixels_dev : FP32 images back to back, image i is [C, H_i, W_i]
 *               (channel, row, column), values as given (normalisation is
 *               applied inside).  The patch grid is floor(H/P) x floor(W/P);
 *               pixels past the last whole patch are ignored.
 *  n_images   : 1 .. 65535.
 *  heights, widths : host arrays; each side >= patch and the grid must have
 *               at most 1024 patches (1025 tokens).
 *  emb_out_dev : [n_images, proj_dim] FP32, each row unit-L2 (norm clamped
 *               at 1e-12).
 *  workspace_dev : >= vl_encode_workspace_bytes(...) bytes, 256-B aligned.
 * All images are packed into one variable-length token stream; attention
 * never crosses images, so each image's result does not depend on what else
 * is in the batch.                                                          */
vl_status vl_encode_images(vl_model* m, const float* pixels_dev,
                           const int32_t* heights, const int32_t* widths,
                           int32_t n_images, float* emb_out_dev,
                           void* workspace_dev, size_t workspace_bytes,
                           void* stream);

/* ---- Contrastive training through the image tower ------------------------
 * Gradients of a training loss with respect to every weight of the image
 * tower, for a caller that forms the loss from the embeddings (for example
 * with vl_contrastive_loss, CLIP Sec. 2.3 / SigLIP Eq. 1, which also returns
 * dL/d(embedding)).  Two calls with the same pixels, shapes and workspace:
 *   vl_encode_images_train    : the encoder forward (bitwise the same
 *                               embeddings as vl_encode_images), keeping in
 *                               the workspace what the backward pass reads;
 *   vl_encode_images_backward : given d_emb_dev [n_images, proj_dim] FP32 =
 *                               dL/d(unit embedding), writes grads_dev, an
 *                               FP32 array of vl_weights_count(cfg) values
 *                               in the weight blob's layout (16-byte
 *                               aligned; overwritten, not accumulated),
 *                               summed over the batch.
 * The backward is the chain rule of each forward step (LayerNorm, GELU,
 * attention, linear layers, patch embedding with the folded pixel
 * normalisation, class token and position table, final LayerNorm, the
 * attention-pooling head with its learned query (VL_POOL_MAP), projection,
 * L2 normalisation).  VL_FP32 models compute in FP32; VL_BF16
 * models multiply BF16 operands (the kept activations, dL/dx of the
 * residual stream, dGELU and dQKV rounded to BF16) with FP32 accumulation;
 * LayerNorm, softmax and L2 statistics stay FP32.
 * Supported: VL_FP32 and VL_BF16 image models, class-token or attention
 * pooling (the latter at head width <= 64; else VL_ERR_UNSUPPORTED), every
 * image at the base patch grid (floor(H/P) ==
 * floor(W/P) == base_grid), at most 2^20 tokens.  The backward returns
 * VL_ERR_INVALID_ARG unless the model's last vl_encode_images_train call had
 * the same pixels pointer, shapes and workspace; the caller must not reuse
 * that workspace in between.  Workspace: vl_train_workspace_bytes(...) bytes,
 * 256-byte aligned (about 2 x (10 D + 2 F) bytes per token per block in BF16,
 * twice that in FP32).  Asynchronous on `stream`.  The first backward call
 * on a VL_BF16 model also allocates (device memory owned by the model, freed
 * by vl_model_destroy) and fills the transposed weights of every block,
 * 2 x L x (4 D^2 + 2 D F) bytes, which later calls reuse; if that
 * allocation fails the call returns VL_ERR_DEVICE.                         */
size_t vl_train_workspace_bytes(const vl_model* m, int32_t n_images, const int32_t* heights,
                                const int32_t* widths);
vl_status vl_encode_images_train(vl_model* m, const float* pixels_dev, const int32_t* heights,
                                 const int32_t* widths, int32_t n_images, float* emb_out_dev,
                                 void* workspace_dev, size_t workspace_bytes, void* stream);
vl_status vl_encode_images_backward(vl_model* m, const float* pixels_dev,
                                    const int32_t* heights, const int32_t* widths,
                                    int32_t n_images, const float* d_emb_dev, float* grads_dev,
                                    void* workspace_dev, size_t workspace_bytes, void* stream);

/* Score unit image embeddings against text embeddings, FP32 throughout.
 *  emb_dev   : [n_images, dim]   texts_dev : [n_texts, dim]  (row-major)
 *  scores_out_dev : [n_images, n_texts] probabilities (softmax over texts)
 *                   or sigmoids of the logits.
 *  top1_out_dev   : [n_images] lowest index attaining the maximum logit, or
 *                   NULL.
 * dim % 4 == 0 and n_texts % 4 == 0 (scores rows are stored 16 bytes at a
 * time); emb, texts and scores 16-byte aligned.  No workspace.             */
vl_status vl_score(const float* emb_dev, int32_t n_images,
                   const float* texts_dev, int32_t n_texts, int32_t dim,
                   vl_head head, float scale, float bias,
                   float* scores_out_dev, int32_t* top1_out_dev,
                   void* stream);

/* Multi-head scaled dot-product attention (Vaswani et al. 2017, Sec. 3.2.1
 * Eq. 1 and Sec. 3.2.2) over packed variable-length sequences: the
 * attention step of vl_encode_images (causal = 0) and vl_encode_texts
 * (causal = 1), exposed on its own with the same kernels.
 *  qkv_dev : [T, 3 * heads * head_dim] token rows [Q | K | V], head k using
 *            columns k*head_dim .. (k+1)*head_dim-1 of each part; BF16 when
 *            prec is VL_BF16, FP32 when VL_FP32; 16-byte aligned.
 *            T = sum of lengths; sequence i occupies the lengths[i] rows
 *            after sequence i-1.
 *  lengths : host array of n_seqs lengths, each 1..4096; 1 <= n_seqs <= 65535.
 *  heads   : 1..64; head_dim: 32 or 64 (else VL_ERR_UNSUPPORTED).
 *  causal  : 0: every token attends to every token of its sequence;
 *            1: token i attends to tokens 0..i of its sequence.
 *  out_dev : [T, heads * head_dim], element type as qkv, 16-byte aligned:
 *            softmax(q k^T / sqrt(head_dim)) v per head, never across
 *            sequences.
 *  workspace_dev : >= vl_attention_workspace_bytes(n_seqs, lengths) bytes,
 *            256-byte aligned (per-sequence descriptors and work items).
 * Softmax maximum and sum are FP32; the BF16 kernel multiplies BF16 Q, K,
 * V and rounds the probabilities to BF16 before the product with V, with
 * FP32 accumulation.  Asynchronous on `stream`; the descriptors are copied
 * from a pinned host buffer the library owns.                              */
size_t vl_attention_workspace_bytes(int32_t n_seqs, const int32_t* lengths);
vl_status vl_attention(const void* qkv_dev, vl_precision prec, const int32_t* lengths,
                       int32_t n_seqs, int32_t heads, int32_t head_dim, int32_t causal,
                       void* out_dev, void* workspace_dev, size_t workspace_bytes,
                       void* stream);

/* Backward of vl_attention without a mask (causal = 0; the image tower's
 * attention), per head h of each sequence (Vaswani et al. 2017, Sec. 3.2.1
 * Eq. 1, differentiated): with S = Q K^T / sqrt(d), P = softmax(S) by rows
 * and O = P V,  dV = P^T dO,  dP = dO V^T,  dS = P * (dP - rowsum(dO * O)),
 *  dQ = dS K / sqrt(d),  dK = dS^T Q / sqrt(d).
 *  qkv_dev   : as for vl_attention ([T, 3 * heads * head_dim], BF16 or FP32).
 *  out_dev   : the forward's output O [T, heads * head_dim] (vl_attention's
 *              out_dev for the same qkv), element type as qkv.
 *  d_out_dev : dL/dO [T, heads * head_dim] FP32.
 *  lengths, n_seqs, heads, head_dim : as for vl_attention.
 *  d_qkv_dev : written, [T, 3 * heads * head_dim] = [dQ | dK | dV] in the
 *              layout of qkv, element type as qkv.
 *  workspace_dev : >= vl_attention_backward_workspace_bytes(n_seqs, lengths,
 *              heads, head_dim) bytes, 256-byte aligned (descriptors, the
 *              per-query log-sum-exp and rowsum(dO * O), dO in BF16).
 * All device pointers 16-byte aligned.  The BF16 kernels recompute P from
 * BF16 Q and K with FP32 softmax statistics, round dO, P and dS to BF16 as
 * matrix operands and accumulate in FP32; FP32 runs FMA kernels throughout.
 * Asynchronous on `stream`; the descriptors are copied from a pinned host
 * buffer the library owns.  The workspace query returns 0 for invalid
 * arguments.                                                               */
size_t vl_attention_backward_workspace_bytes(int32_t n_seqs, const int32_t* lengths,
                                             int32_t heads, int32_t head_dim);
vl_status vl_attention_backward(const void* qkv_dev, const void* out_dev,
                                const float* d_out_dev, vl_precision prec,
                                const int32_t* lengths, int32_t n_seqs, int32_t heads,
                                int32_t head_dim, void* d_qkv_dev, void* workspace_dev,
                                size_t workspace_bytes, void* stream);

/* Contrastive loss of n matched (image, text) pairs, e.g. the embeddings of
 * a training batch, and its gradient.  Logits l_ij = scale <e_i, t_j> + bias;
 *  VL_HEAD_SOFTMAX (CLIP, Radford et al. 2021, Sec. 2.3): L = the mean of
 *    the image->text and text->image cross-entropies, target = the matching
 *    pair (bias has no effect; its gradient is 0);
 *  VL_HEAD_SIGMOID (SigLIP, Zhai et al. 2023, Eq. 1):
 *    L = -(1/n) sum_ij log sigmoid(z_ij l_ij), z_ij = +1 if i == j else -1.
 * Inputs emb_dev, texts_dev [n, dim] FP32 (any vectors; not normalised
 * here).  Outputs (device): loss_dev[1]; d_emb_dev, d_texts_dev [n, dim] =
 * dL/de, dL/dt; d_scale_bias_dev[2] = (dL/dscale, dL/dbias).  FP32
 * throughout, deterministic.  dim % 16 == 0, 1 <= n <= 65535, scale > 0;
 * arrays 16-byte aligned, workspace >= vl_contrastive_workspace_bytes(n,
 * dim) bytes, 256-byte aligned (about 8 n^2 bytes).                         */
size_t vl_contrastive_workspace_bytes(int32_t n, int32_t dim);
vl_status vl_contrastive_loss(const float* emb_dev, const float* texts_dev, int32_t n,
                              int32_t dim, vl_head head, float scale, float bias,
                              float* loss_dev, float* d_emb_dev, float* d_texts_dev,
                              float* d_scale_bias_dev, void* workspace_dev,
                              size_t workspace_bytes, void* stream);

/* Allocation-free variant of vl_contrastive_loss, for callers that cannot
 * allocate device memory or pass a workspace: code under HIP graph capture,
 * tight training or serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels, results (bitwise) and errors as vl_contrastive_loss,
 * minus the workspace: the kernels' scratch (logits, their transpose, the
 * transposed embeddings, per-row partials) lives in a static device array of
 * VL_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until the
 * process ends.  Its device address is looked up once per device on the
 * first call made with that device current.  The call allocates nothing
 * (no hipMalloc / hipFree, no pinned memory, no events) and enqueues only
 * kernels on `stream`.  Requires vl_contrastive_workspace_bytes(n, dim) <=
 * VL_NOALLOC_SCRATCH_BYTES (n <= 2528 at dim 768, 2422 at dim 1024), else
 * VL_ERR_WORKSPACE_TOO_SMALL with nothing enqueued.  Every call on one GPU
 * shares that GPU's array and overwrites it (nothing in it needs to start
 * at zero): calls that overlap on one GPU, i.e. are in flight at the same
 * time on different streams, race and give undefined results; serialise
 * them on one stream or order them with events.                            */
#define VL_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
vl_status vl_contrastive_loss_noalloc(const float* emb_dev, const float* texts_dev, int32_t n,
                                      int32_t dim, vl_head head, float scale, float bias,
                                      float* loss_dev, float* d_emb_dev, float* d_texts_dev,
                                      float* d_scale_bias_dev, void* stream);

/* The number-format conversions of the reduced-precision paths, exposed so
 * callers can prepare operands and check them.
 * vl_bf16_round: FP32 -> BF16, round to nearest, ties to even, on n values
 *   (n > 0, even; src 8-byte, dst 4-byte aligned; dst receives BF16 bit
 *   patterns).  method 0: the integer rounding of the FP32 bit pattern
 *   (add 0x7FFF plus the lowest kept bit, drop 16 bits) that the LayerNorm,
 *   weight conversion and single-value stores use; method 1: the gfx950
 *   packed conversion instruction (v_cvt_pk_bf16_f32) of the GEMM epilogues
 *   and attention probabilities.  Finite inputs round identically; NaN
 *   payloads are not specified.
 * vl_fp8_quantize_rows: the VL_FP8W_BF16A weight quantiser on FP32 rows
 *   [rows, cols]: scales[r] = max_c |src[r][c]| / 448 (1 for an all-zero
 *   row), codes[r][c] = OCP e4m3fn code of src[r][c] / scales[r], rounded to
 *   nearest even, saturating at +-448 (OFP8 rev 1.0, Sec. 5.1).           */
vl_status vl_bf16_round(const float* src_dev, int64_t n, int32_t method, uint16_t* dst_dev,
                        void* stream);
vl_status vl_fp8_quantize_rows(const float* src_dev, int32_t rows, int32_t cols,
                               uint8_t* codes_dev, float* scales_dev, void* stream);

/* MXFP8 encoding (the one VL_MXFP8 applies to its weights and activations)
 * of FP32 rows, for callers that prepare operands themselves and for
 * checking the encoder.
 *  src_dev    : [rows, cols] FP32, row-major, 16-byte aligned.
 *  codes_dev  : [rows, cols] e4m3 codes (OFP8 rev 1.0, Sec. 5.1), 4-byte
 *               aligned.
 *  scales_dev : (cols/128) * rows * 4 E8M0 bytes (value 2^(byte - 127)),
 *               block-major: the scale of row r, columns 32j .. 32j+31 is
 *               byte (j/4 * rows + r) * 4 + s(j % 4) with s = {0, 2, 1, 3}.
 * cols % 128 == 0, rows > 0.  Values must be finite.                      */
vl_status vl_mx_quantize(const float* src_dev, int32_t rows, int32_t cols,
                         uint8_t* codes_dev, uint8_t* scales_dev, void* stream);

/* The MXFP8 contraction of the VL_MXFP8 model's block linears, exposed on
 * its own:  C[m, n] += sum_k A[m, k] B[n, k] + bias[n]  (FP32 C).
 *  a_dev, b_dev   : e4m3 codes [M, K] and [N, K], row-major, 16-byte aligned.
 *  sa_dev, sb_dev : their E8M0 scales in the layout vl_mx_quantize writes
 *                   ((K/128) * M * 4 and (K/128) * N * 4 bytes), 4-byte
 *                   aligned.  A[m, k] = value(code) * 2^(scale - 127).
 *  bias_dev [N], c_dev [M, N] : FP32, 16-byte aligned; c is read and written.
 *  cfg : -1 (heuristic) or an MXFP8 tile configuration id (name "MX_...").
 * K % 128 == 0, N % 32 == 0.  The products are summed by the gfx950 scaled
 * FP8 MFMA (64 values of K per instruction) into FP32 accumulators, K in
 * ascending order, the same in every configuration.                        */
vl_status vl_mx_gemm(const uint8_t* a_dev, const uint8_t* sa_dev, const uint8_t* b_dev,
                     const uint8_t* sb_dev, int32_t M, int32_t N, int32_t K,
                     const float* bias_dev, float* c_dev, int32_t cfg, void* stream);

const char* vl_status_string(vl_status s);
const char* vl_last_error_message(void);
int32_t vl_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VL_H_ */
