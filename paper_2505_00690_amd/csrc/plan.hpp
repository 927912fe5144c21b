// Host-side planning of an encode call: how a packed batch of images (or
// token sequences) is cut into parts, which attention work items and
// descriptors the kernels read, and where every activation buffer sits in
// the caller's workspace.  Plain C++ (no device code or HIP calls), so it
// also builds on its own for host-only checks.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "batch.hpp"

namespace vl {

constexpr size_t kAlign = 256;     // workspace and region alignment
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

constexpr int kMaxTokens = 1025;   // 32 x 32 patches + class token
constexpr int kAttnQ = 128;        // queries per attention work item
constexpr int kResMinTokens = 128; // K/V-resident attention: more tokens than one work item
constexpr int kResMaxTiles = 10;   //   and at most 10 key tiles of 64 (the 160 KB of LDS)
constexpr int kMaxItems = 65535;   // images / texts per call (grid y of the gather kernels)
constexpr int64_t kSplitMinTokens = 4096;  // two-part batches from this many tokens
constexpr int64_t kMaxBatchTokens = int64_t(1) << 24;

// What planning needs to know of a model.
struct PlanModel {
  bool text = false;          // sequences of token ids (else images)
  bool split = false;         // two-part batches allowed (option on, not FP32)
  bool resident = false;      // K/V-resident attention usable (option on, BF16 or MXFP8
                              // activations, head width 64, image model)
  bool map_pool = false;      // attention-pooling head buffers
  bool fold_buffers = false;  // LayerNorm folding buffers (BF16 / e4m3-weight models)
  int es = 2;                 // bytes per activation element (4 for FP32 models)
  int D = 0, F = 0, Kpad = 0, Pd = 0;  // width, MLP width, padded patch length, output dim
  int P = 1, channels = 3;    // patch side and input planes (images)
  int ctx = 0;                // longest sequence (texts)
};

// A batch runs as one or two parts.  A part is a run of consecutive images
// with its own descriptors (token starts relative to the part) and its own
// regions of every activation buffer, so two parts never share memory and
// can run concurrently on two streams.  Every kernel works per token row or
// per image with a fixed accumulation order, so a part computes exactly what
// the whole batch would for its images.
struct Part {
  int i0 = 0, n = 0, T = 0, max_ntok = 0, n_items = 0;
  size_t off_imgs = 0, off_items = 0;                       // in the descriptor region
  // Images whose attention runs K/V-resident (indices within the part) and
  // the largest of their key-tile counts.
  size_t off_res = 0;
  int n_res = 0, res_tiles = 0;
  size_t off_tok = 0, off_X = 0, off_Y = 0, off_QH = 0, off_E = 0;  // in the workspace
  size_t off_map = 0;   // MAP pooling: per image O, x, LN(x) [n, D] and MLP hidden [n, F]
  // LayerNorm folding: u = bf16(x * gamma) [T, D], per-32-column (mean, M2)
  // partials [T, D/32, 2] and row (mean, rstd) [T, 2]
  size_t off_U = 0, off_PS = 0, off_RS = 0;
  // Launch sizes and buffer regions.  Equal to the counts above, except in
  // a bucketed plan, where they are the bucket's capacities and the kernels
  // read the live counts from the part's BatchCounts record at off_bc.
  bool bucketed = false;
  int T_cap = 0, n_cap = 0, items_cap = 0, res_cap = 0, ntok_cap = 0, res_class = 0;
  size_t off_bc = 0;
};

struct Plan {
  bool bucketed = false;
  int n = 0, T = 0;
  std::vector<int32_t> hw;          // (H, W) per image, for graph keys
  std::vector<char> desc;           // host image of the descriptor region
  size_t desc_bytes = 0;
  std::vector<Part> parts;
  size_t total = 0;                 // workspace bytes
};

// Capacities of a bucketed plan.  Tokens: up to 16 as they are; above,
// rounded up to a multiple of 2^(floor(log2 T) - 2) but kept below the next
// power of two, so a bucket spans at most a quarter of its values and the
// capacity has the floor(log2) of the count, which is what the GEMM tile
// choice depends on.  Images: the next power of two (at most kMaxItems).
int cap_tokens(int T);
int cap_images(int n);

// An image batch: n images of heights hs[i] x widths ws[i].  one_part keeps
// it in one part; bucketed sizes the parts for their capacity buckets.
// False (with *why) on invalid input.
bool make_plan(const PlanModel& m, int32_t n, const int32_t* hs, const int32_t* ws, Plan* p,
               std::string* why, bool one_part = false, bool bucketed = false);

// A text batch: n sequences of lens[i] tokens; descriptors hold the
// sequence's offset in the packed id stream and graph keys (length, 0).
bool make_text_plan(const PlanModel& m, int32_t n, const int32_t* lens, Plan* p,
                    std::string* why);

// A bucketed plan's per-call pointers: the pixel buffer and each part's
// first output row, written into the parts' BatchCounts records.
void bind_batch(Plan& p, const void* pix, float* emb, int Pd);

}  // namespace vl
